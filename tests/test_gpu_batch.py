"""tk_compress_batch: problems of uneven sizes run concurrently on the context's worker
streams; every result must be identical to what tk_compress returns for the problem alone,
also when a small HBM budget makes the problems wait for admission."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    from paper_1711_06874_amd import tk as mod
    return mod


# (n, nu, ell, layout): uneven sizes, all three Matern orders, both layouts
_ITEMS = [(48, 0.5, 0.1, 1), (33, 1.5, 0.3, 0), (64, 2.5, 1.0, 1), (40, 0.5, 0.3, 1),
          (57, 1.5, 0.1, 0), (32, 2.5, 0.3, 1), (64, 0.5, 1.0, 0)]


def _problems(tk):
    ks = [tk.make_kernel(0, nu=nu, ell=ell) for (_, nu, ell, _) in _ITEMS]
    gs = [tk.make_grid(n, 1.0, lay) for (n, _, _, lay) in _ITEMS]
    return ks, gs


def _same(a, b):
    (Ua, Ca), (Ub, Cb) = a.factors(), b.factors()
    return (a.ranks == b.ranks and a.rel_err == b.rel_err and np.array_equal(Ca, Cb)
            and all(np.array_equal(x, y) for x, y in zip(Ua, Ub)))


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batch_matches_single(tk, prec):
    require_gpu()
    ctx = tk.Context(0)
    try:
        ks, gs = _problems(tk)
        opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
        alone = [ctx.compress(k, g, opts) for k, g in zip(ks, gs)]
        for workers in (4, 2):
            ctx.set_workers(workers)
            say("batch prec", prec, "workers", workers)
            mix = ctx.compress_batch(ks, gs, opts)
            for i, (a, b) in enumerate(zip(alone, mix)):
                assert _same(a, b), f"item {i} differs in the batch"
            for t in mix:
                t.free()
        for t in alone:
            t.free()
    finally:
        ctx.destroy()


def test_batch_under_tight_budget(tk):
    """A budget that holds about one problem at a time: the others wait, nothing fails."""
    require_gpu()
    ks, gs = _problems(tk)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=1)
    big = tk.tk_estimate_bytes(gs[2], opts)
    ctx = tk.Context(0, hbm_budget_bytes=int(1.5 * big))
    try:
        alone = [ctx.compress(k, g, opts) for k, g in zip(ks, gs)]
        ref = [(t.ranks, t.rel_err, t.factors()) for t in alone]
        for t in alone:
            t.free()
        mix = ctx.compress_batch(ks, gs, opts)
        for i, (t, (r, e, (U, C))) in enumerate(zip(mix, ref)):
            Ub, Cb = t.factors()
            assert t.ranks == r and t.rel_err == e and np.array_equal(Cb, C), f"item {i}"
            assert all(np.array_equal(x, y) for x, y in zip(U, Ub)), f"item {i}"
        for t in mix:
            t.free()
    finally:
        ctx.destroy()


def test_batch_empty_and_errors(tk):
    require_gpu()
    ctx = tk.Context(0)
    try:
        assert ctx.compress_batch([], [], tk.make_opts(eps=1e-6)) == []
        ks, gs = _problems(tk)
        bad = list(ks)
        bad[3] = tk.make_kernel(0, nu=31.0, ell=0.3)       # unsupported order (above 30)
        with pytest.raises(tk.TkError) as ei:
            ctx.compress_batch(bad, gs, tk.make_opts(eps=1e-6))
        assert ei.value.status == tk.TK_EUNSUPPORTED
        with pytest.raises(tk.TkError):
            ctx.set_workers(0)
    finally:
        ctx.destroy()


# problems on shared grids: 34 on the 33^3 centred grid (two launches of 17), 3 on the 48^3
# offset grid (one launch of 3), one alone
def _grouped(tk):
    rng = np.random.default_rng(5)
    items = [(33, 0)] * 34 + [(48, 1)] * 3 + [(40, 1)]
    ks = [tk.make_kernel(0, nu=float(rng.choice([0.5, 1.5, 2.5])), ell=float(np.exp(rng.uniform(np.log(0.05), 0.0))))
          for _ in items]
    gs = [tk.make_grid(n, 1.0, lay) for (n, lay) in items]
    return ks, gs


@pytest.mark.parametrize("prec,eps,ranks", [(1, 1e-6, (0, 0, 0)), (2, 1e-6, (0, 0, 0)), (1, 0.0, (5, 6, 7)),
                                            (0, 0.0, (4, 4, 6)), (0, 1e-6, (0, 0, 0))])
def test_grouped_batch_matches_single(tk, prec, eps, ranks):
    """Problems on one grid share every launch (grid z over the problems); each result is
    bitwise the one the problem gets alone.  The FP64 eps path (ranks read back between steps)
    runs its problems one per call."""
    require_gpu()
    ctx = tk.Context(0)
    try:
        ks, gs = _grouped(tk)
        opts = tk.make_opts(eps=eps, ranks=ranks, hooi_sweeps=2, prec=prec)
        say("grouped batch prec", prec, "eps", eps, "ranks", ranks)
        alone = [ctx.compress(k, g, opts, allow_noconv=True) for k, g in zip(ks, gs)]
        for workers in (4, 1):
            ctx.set_workers(workers)
            mix = ctx.compress_batch(ks, gs, opts)
            for i, (a, b) in enumerate(zip(alone, mix)):
                assert _same(a, b), f"item {i} differs in the batch"
            for t in mix:
                t.free()
        for t in alone:
            t.free()
    finally:
        ctx.destroy()


def test_grouped_batch_budget_caps_launch_size(tk):
    """A budget of about 2.5 problems: a shared-grid group is split into launches that fit."""
    require_gpu()
    ks, gs = _grouped(tk)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=1)
    per = tk.tk_estimate_bytes(gs[0], opts)
    ctx = tk.Context(0, hbm_budget_bytes=int(2.5 * max(per, tk.tk_estimate_bytes(gs[34], opts))))
    try:
        ref = []
        for k, g in zip(ks, gs):
            t = ctx.compress(k, g, opts)
            ref.append((t.ranks, t.rel_err, t.factors()))
            t.free()
        mix = ctx.compress_batch(ks, gs, opts)
        for i, (t, (r, e, (U, C))) in enumerate(zip(mix, ref)):
            Ub, Cb = t.factors()
            assert t.ranks == r and t.rel_err == e and np.array_equal(Cb, C), f"item {i}"
            assert all(np.array_equal(x, y) for x, y in zip(U, Ub)), f"item {i}"
        for t in mix:
            t.free()
    finally:
        ctx.destroy()


def test_concurrent_large_n_matches_single(tk):
    """Sizes above 64 put eigensolver rows in every wave of a work-group, and concurrent
    launches on other streams shift the waves' timing: results must still be bitwise those of
    the problems alone (shared-grid groups and single problems, 4 and 8 workers)."""
    require_gpu()
    rng = np.random.default_rng(11)
    sizes = [96] * 6 + [128] * 6 + [160, 112, 144, 100]
    ks = [tk.make_kernel(0, nu=float(rng.choice([0.5, 1.5, 2.5])), ell=float(np.exp(rng.uniform(np.log(0.05), 0.0))))
          for _ in sizes]
    gs = [tk.make_grid(n, 1.0, 0) for n in sizes]
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=1)
    ctx = tk.Context(0)
    try:
        ref = []
        for k, g in zip(ks, gs):
            t = ctx.compress(k, g, opts)
            ref.append((t.ranks, t.rel_err, t.factors()))
            t.free()
        for workers in (4, 8):
            ctx.set_workers(workers)
            for rep in range(2):
                say("concurrent large n, workers", workers, "rep", rep)
                mix = ctx.compress_batch(ks, gs, opts)
                for i, (t, (r, e, (U, C))) in enumerate(zip(mix, ref)):
                    Ub, Cb = t.factors()
                    assert t.ranks == r and t.rel_err == e and np.array_equal(Cb, C), f"item {i} (n={sizes[i]})"
                    assert all(np.array_equal(x, y) for x, y in zip(U, Ub)), f"item {i} (n={sizes[i]})"
                for t in mix:
                    t.free()
    finally:
        ctx.destroy()


def test_autotune_keeps_batch_equal_single_and_roundtrips(tk, tmp_path):
    """Tuned Gram split counts apply to single and batched calls alike (bitwise equal), meet eps,
    and a saved table gives a second context the same results."""
    require_gpu()
    g = tk.make_grid(96, 1.0, 1)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=1)
    ks = [tk.make_kernel(0, nu=nu, ell=ell) for nu, ell in [(0.5, 0.1), (1.5, 0.3), (2.5, 0.6), (1.5, 0.05)]]
    ctx = tk.Context(0)
    try:
        for prec in (1, 2):
            r = ctx.autotune(g, prec)
            say("autotune prec", prec, r)
            assert all(s >= 1 for s in r["nsplit"]) and all(m > 0 for m in r["ms"])
        ref = []
        for k in ks:
            t = ctx.compress(k, g, opts)
            assert t.rel_err <= 1e-6
            ref.append((t.ranks, t.rel_err, t.factors()))
            t.free()
        mix = ctx.compress_batch(ks, [g] * len(ks), opts)
        for i, (t, (rk, e, (U, C))) in enumerate(zip(mix, ref)):
            Ub, Cb = t.factors()
            assert t.ranks == rk and t.rel_err == e and np.array_equal(Cb, C), f"item {i}"
            assert all(np.array_equal(x, y) for x, y in zip(U, Ub)), f"item {i}"
            t.free()
        path = tmp_path / "tune.json"
        ctx.autotune_save(str(path))
        bad = tmp_path / "bad.json"
        bad.write_text('{"format": "tk-autotune-1", "entries": [{"n": [96, 96], "mode": 0}]}')
        ctx2 = tk.Context(0)
        try:
            with pytest.raises(tk.TkError):
                ctx2.autotune_load(str(bad))
            ctx2.autotune_load(str(path))
            for k, (rk, e, (U, C)) in zip(ks, ref):
                t = ctx2.compress(k, g, opts)
                Ub, Cb = t.factors()
                assert t.ranks == rk and t.rel_err == e and np.array_equal(Cb, C)
                t.free()
        finally:
            ctx2.destroy()
    finally:
        ctx.destroy()


def test_graph_replay_matches_direct_launches(tk):
    """With graph replay on, the first call of a shape captures the pipeline and later calls
    replay it with the sampling launch updated to their own kernels and grids: every replay,
    with direct-launch work of the same context in between, gives bitwise the direct result
    (single calls, shared-grid groups, concurrent batches, fixed ranks and eps truncation)."""
    require_gpu()
    rng = np.random.default_rng(23)
    ks = [tk.make_kernel(0, nu=float(rng.choice([0.5, 1.5, 2.5])), ell=float(np.exp(rng.uniform(np.log(0.05), 0.0))))
          for _ in range(6)]
    # same sizes, different extents and layouts: the replayed graph must take the call's grid
    gs = [tk.make_grid(48, 1.0, 1), tk.make_grid(48, 0.5, 0), tk.make_grid(48, 2.0, 1),
          tk.make_grid(96, 1.0, 0), tk.make_grid(48, 1.0, 0), tk.make_grid(96, 0.7, 1)]
    for prec, eps, ranks in [(1, 1e-6, (0, 0, 0)), (2, 1e-6, (0, 0, 0)), (0, 0.0, (4, 5, 6))]:
        opts = tk.make_opts(eps=eps, ranks=ranks, hooi_sweeps=2, prec=prec)
        ctx = tk.Context(0)
        try:
            alone = [ctx.compress(k, g, opts, allow_noconv=True) for k, g in zip(ks, gs)]
            group_ref = ctx.compress_group(ks[:3], gs[0], opts)
            ctx.set_graphs(True)
            for rep in range(3):
                say("graph replay prec", prec, "eps", eps, "rep", rep)
                for i, (k, g) in enumerate(zip(ks, gs)):
                    t = ctx.compress(k, g, opts, allow_noconv=True)
                    assert _same(t, alone[i]), f"single {i} differs on replay {rep}"
                    t.free()
                grp = ctx.compress_group(ks[:3], gs[0], opts)
                for i, (a, b) in enumerate(zip(group_ref, grp)):
                    assert _same(a, b), f"group item {i} differs on replay {rep}"
                for t in grp:
                    t.free()
                mix = ctx.compress_batch(ks, gs, opts)
                for i, (a, b) in enumerate(zip(alone, mix)):
                    assert _same(a, b), f"batch item {i} differs on replay {rep}"
                for t in mix:
                    t.free()
                # direct launches between the replays
                ctx.set_graphs(False)
                t = ctx.compress(ks[rep], gs[rep], opts, allow_noconv=True)
                assert _same(t, alone[rep])
                t.free()
                ctx.set_graphs(True)
            for t in alone + group_ref:
                t.free()
        finally:
            ctx.destroy()


@pytest.mark.parametrize("prec", [1, 2])
def test_uneven_batch_grids_in_one_persistent_launch(tk, prec):
    """Float batches of uneven sizes evaluate every grid in one persistent launch (work items
    of all sizes taken from a device counter) into the workspace laid out for all units at
    once; the results stay bitwise those of single calls."""
    require_gpu()
    ctx = tk.Context(0)
    try:
        ks, gs = _problems(tk)
        opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
        alone = [ctx.compress(k, g, opts) for k, g in zip(ks, gs)]
        tk.tk_profile_reset()
        tk.tk_profile_select(["grid"])
        tk.tk_profile_enable(True)
        mix = ctx.compress_batch(ks, gs, opts)
        tk.tk_profile_enable(False)
        launches, ms = tk.tk_profile_read(tk.PROF_CLASSES["grid"])
        tk.tk_profile_reset()
        tk.tk_profile_select(None)
        say("grid launches in the batch: %d (%.3f ms)" % (launches, ms))
        assert launches == 1
        for i, (a, b) in enumerate(zip(alone, mix)):
            assert _same(a, b), f"item {i} differs in the batch"
        for t in mix + alone:
            t.free()
    finally:
        ctx.destroy()
