"""GPU: the batched executor (h1w_batch_solve) over independent GN systems of
uneven size, checked item by item against the CPU oracle's FP64 true residual
and against single-instance solves of the same systems."""
import numpy as np
import pytest

import h1w_inputs as H
from oracle import gn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2209_02815_amd as P
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def small_batch():
    # uneven 2D instances plus one 3D instance and one without rows
    wls = H.batch_workloads(count=10, batch_id=7, sides=(17, 33, 65), m_lo=1, m_hi=40)
    wls.append(H.workload("cube17").with_(name="b3d", wid=700011, alpha=3e-4, m=11))
    wls.append(H.workload("square33").with_(name="b0", wid=700012, m=0))
    return wls


def make_items(wls):
    items, host = [], []
    for wl in wls:
        J = H.j_rows(wl) if wl.m > 0 else None
        b = H.rhs_b(wl)
        items.append(dict(shape=wl.shape, beta=wl.beta, alpha=wl.alpha, J=None if J is None else dev(J),
                          b=dev(b), x=torch.zeros(wl.N, dtype=torch.float64, device="cuda:0")))
        host.append((J, b))
    return items, host


@pytest.mark.parametrize("prec,rtol,nworkers", [("fp64", 1e-10, 4), ("mixed", 1e-8, 3), ("fp64", 1e-10, 1)])
def test_batch_matches_oracle(P, prec, rtol, nworkers):
    from paper_2209_02815_amd import _native as nat
    wls = small_batch()
    items, host = make_items(wls)
    precision = nat.H1W_FP64 if prec == "fp64" else nat.H1W_MIXED
    infos, stats, rep = nat.h1w_batch_solve(items, precision=precision, nworkers=nworkers, rtol=rtol)
    assert all(s == 0 for s in stats) and rep.nworkers == nworkers and rep.t_total_ms > 0
    for wl, it, (J, b), info in zip(wls, items, host, infos):
        x = it["x"].cpu().numpy()
        Jm = J if J is not None else np.zeros((0, wl.N))
        rr = gn.true_relres(wl.shape, wl.beta, Jm, wl.alpha, b, x)
        assert rr <= 1.01 * rtol, (wl.name, rr, info.as_dict())
        floor = gn.residual_rounding_floor(wl.shape, wl.beta, Jm, wl.alpha, b, x)
        assert abs(rr - info.relres_true) <= 1e-3 * rtol + floor


def test_batch_equals_single_solves(P):
    # the executor runs the library's own solve: same iterations and the same
    # solution as one-at-a-time calls on the same grid settings
    from paper_2209_02815_amd import _native as nat
    wls = small_batch()[:6]
    items, host = make_items(wls)
    infos, stats, _ = nat.h1w_batch_solve(items, nworkers=4, rtol=1e-10)
    assert all(s == 0 for s in stats)
    for wl, it, info in zip(wls, items, infos):
        with P.Context(wl.shape, wl.beta) as ctx:
            x, si = ctx.gn_solve(it["J"], wl.alpha, b=it["b"], rtol=1e-10)
        assert si.iters == info.iters
        xb = it["x"].cpu().numpy()
        xs = x.cpu().numpy()
        assert np.linalg.norm(xb - xs) <= 1e-12 * np.linalg.norm(xs)


def test_batch_autotune_reports_choices(P):
    from paper_2209_02815_amd import _native as nat
    wls = H.batch_workloads(count=14, batch_id=8, sides=(33, 65), m_lo=20, m_hi=30)
    items, host = make_items(wls)
    infos, stats, rep = nat.h1w_batch_solve(items, nworkers=2, autotune=2, rtol=1e-10)   # tune every key
    assert all(s == 0 for s in stats)
    # one key per grid (the smoother schedule changes B, not J)
    tuned = [rep.tuned[k] for k in range(rep.ntuned)]
    assert {t.n[0] for t in tuned} == {wl.shape[0] for wl in wls} and len(tuned) == 2
    assert all(t.nu == 2 and t.ms_per_unit > 0 and t.reused == 0 for t in tuned)
    # an interval other than the default is chosen only with fewer CG iterations
    for t in tuned:
        assert t.cheb_lo in (0.3, 0.4, 0.5)
        assert 0 < t.iters <= t.iters_default
        assert (t.cheb_lo == 0.3) == (t.iters == t.iters_default), (t.cheb_lo, t.iters, t.iters_default)
    chosen = {t.n[0]: t.cheb_lo for t in tuned}
    print("tuned lower Chebyshev bounds:", chosen, [(t.iters, t.iters_default) for t in tuned], flush=True)
    # a second batch of the process reuses the choices (autotune = 1)
    _, stats2, rep2 = nat.h1w_batch_solve(items, nworkers=2, autotune=1, rtol=1e-10)
    assert all(s == 0 for s in stats2)
    assert all(rep2.tuned[k].reused == 1 for k in range(rep2.ntuned))
    assert {rep2.tuned[k].n[0]: rep2.tuned[k].cheb_lo for k in range(rep2.ntuned)} == chosen
    for wl, it, (J, b) in zip(wls, items, host):
        rr = gn.true_relres(wl.shape, wl.beta, J, wl.alpha, b, it["x"].cpu().numpy())
        assert rr <= 1.01e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_autotune_departs_where_iterations_drop(P, prec):
    # on 129^2 grids at rtol 1e-8 the Chebyshev interval [0.4, 2] or [0.5, 2]
    # needs one CG iteration fewer than the default [0.3, 2]: the tuner must
    # take it (its choice rests on iteration counts, so it is deterministic),
    # and every instance solved with it must still meet the tolerance
    from paper_2209_02815_amd import _native as nat
    wls = H.batch_workloads(count=6, batch_id=9, sides=(129,), m_lo=40, m_hi=60)
    items, host = make_items(wls)
    precision = {"fp64": nat.H1W_FP64, "mixed": nat.H1W_MIXED}[prec]
    infos, stats, rep = nat.h1w_batch_solve(items, precision=precision, nworkers=2, autotune=2, rtol=1e-8)
    assert all(s == 0 for s in stats)
    assert rep.ntuned == 1
    t = rep.tuned[0]
    print(f"{prec}: chosen lower bound {t.cheb_lo}, iterations {t.iters} against {t.iters_default}", flush=True)
    assert t.cheb_lo in (0.4, 0.5) and t.iters < t.iters_default
    for wl, it, (J, b) in zip(wls, items, host):
        rr = gn.true_relres(wl.shape, wl.beta, J, wl.alpha, b, it["x"].cpu().numpy())
        assert rr <= 1.01e-8


@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-10), ("fp64", 1e-8), ("mixed", 1e-8)])
def test_grouped_batch_matches_oracle(P, prec, rtol):
    # lock-step mode: every instance of a grid advanced together; each x must
    # meet rtol on the oracle's FP64 true residual, as the reported one says
    from paper_2209_02815_amd import _native as nat
    wls = small_batch() + H.batch_workloads(count=6, batch_id=11, sides=(65,), m_lo=100, m_hi=128)
    items, host = make_items(wls)
    precision = {"fp64": nat.H1W_FP64, "mixed": nat.H1W_MIXED}[prec]
    infos, stats, rep = nat.h1w_batch_solve(items, precision=precision, nworkers=3, rtol=rtol, grouped=True)
    assert all(s == 0 for s in stats)
    worst = 0.0
    for wl, it, (J, b), inf in zip(wls, items, host, infos):
        x = it["x"].cpu().numpy()
        Jm = J if J is not None else np.zeros((0, wl.N))
        rr = gn.true_relres(wl.shape, wl.beta, Jm, wl.alpha, b, x)
        floor = gn.residual_rounding_floor(wl.shape, wl.beta, Jm, wl.alpha, b, x)
        assert rr <= 1.01 * rtol, (wl.name, rr)
        assert abs(rr - inf.relres_true) <= 1e-3 * rtol + floor, (wl.name, rr, inf.relres_true)
        worst = max(worst, rr)
    print(f"grouped {prec} rtol {rtol}: worst true residual {worst:.2e}, iterations "
          f"{sorted(i.iters for i in infos)}", flush=True)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_grouped_batch_autotune_departs_where_iterations_drop(P, prec):
    # the grouped mode solves the whole group with each schedule and keeps
    # the one with the least work (iterations weighted by m + 1): on 129^2
    # grids at rtol 1e-8 that is [0.4, 2] or [0.5, 2], one CG iteration fewer
    # than the default for every instance of the group, each of which must
    # still meet the tolerance on the oracle's true residual
    from paper_2209_02815_amd import _native as nat
    wls = H.batch_workloads(count=6, batch_id=9, sides=(129,), m_lo=40, m_hi=60)
    items, host = make_items(wls)
    precision = {"fp64": nat.H1W_FP64, "mixed": nat.H1W_MIXED}[prec]
    infos0, stats0, _ = nat.h1w_batch_solve(items, precision=precision, nworkers=1, autotune=0, rtol=1e-8,
                                            grouped=True)
    assert all(s == 0 for s in stats0)
    iters0 = [i.iters for i in infos0]
    infos, stats, rep = nat.h1w_batch_solve(items, precision=precision, nworkers=1, autotune=2, rtol=1e-8,
                                            grouped=True)
    assert all(s == 0 for s in stats)
    assert rep.ntuned == 1
    t = rep.tuned[0]
    iters = [i.iters for i in infos]
    print(f"grouped {prec}: chosen lower bound {t.cheb_lo}, group iterations {t.iters} against "
          f"{t.iters_default}; per instance {iters} against {iters0}", flush=True)
    assert t.grouped == 1
    assert t.cheb_lo in (0.4, 0.5) and t.iters < t.iters_default
    assert t.iters == sum(iters) and t.iters_default == sum(iters0)
    assert sum(iters) < sum(iters0)
    for wl, it, (J, b) in zip(wls, items, host):
        rr = gn.true_relres(wl.shape, wl.beta, J, wl.alpha, b, it["x"].cpu().numpy())
        assert rr <= 1.01e-8
    # a later batch reuses the choice (autotune = 1) without tuning again
    infos2, stats2, rep2 = nat.h1w_batch_solve(items, precision=precision, nworkers=1, autotune=1, rtol=1e-8,
                                               grouped=True)
    assert all(s == 0 for s in stats2)
    assert rep2.ntuned == 1 and rep2.tuned[0].reused == 1 and rep2.tuned[0].cheb_lo == t.cheb_lo
    assert [i.iters for i in infos2] == iters


def test_grouped_batch_cut_groups_and_zero_rhs(P):
    # 300 instances on one grid are cut into groups of at most 256 (two
    # groups, so two workers solve the same grid at once); an instance with
    # b = 0 never becomes active and returns x = 0 exactly
    from paper_2209_02815_amd import _native as nat
    wls = H.batch_workloads(count=300, batch_id=14, sides=(17,), m_lo=1, m_hi=8)
    items, host = make_items(wls)
    zero = 7
    items[zero]["b"].zero_()
    infos, stats, rep = nat.h1w_batch_solve(items, nworkers=2, rtol=1e-10, grouped=True)
    assert all(s == 0 for s in stats)
    assert rep.nworkers == 2
    assert torch.count_nonzero(items[zero]["x"]).item() == 0
    assert infos[zero].iters == 0 and infos[zero].relres_true == 0.0
    for k, (wl, it, (J, b)) in enumerate(zip(wls, items, host)):
        if k == zero:
            continue
        rr = gn.true_relres(wl.shape, wl.beta, J, wl.alpha, b, it["x"].cpu().numpy())
        assert rr <= 1.01e-10, (k, rr)


def test_grouped_batch_failures_stay_with_their_items(P):
    # with maxit below what some instances need, those instances end ENOCONV
    # and the rest of their group is solved as usual; an instance whose b holds
    # a NaN ends ENUMERIC without touching the others
    from paper_2209_02815_amd import _native as nat
    wls = small_batch() + H.batch_workloads(count=6, batch_id=11, sides=(65,), m_lo=100, m_hi=128)
    items, host = make_items(wls)
    ref, _, _ = nat.h1w_batch_solve(items, nworkers=2, rtol=1e-8, grouped=True)
    need = [i.iters for i in ref]
    cap = sorted(need)[len(need) // 2]
    assert max(need) > cap
    bad = 3
    items[bad]["b"][5] = float("nan")
    for it in items:
        it["x"].zero_()
    infos, stats, rep = nat.h1w_batch_solve(items, nworkers=2, rtol=1e-8, maxit=cap, grouped=True,
                                            raise_on_error=False)
    assert stats[bad] == nat.H1W_ENUMERIC
    n_ok = n_fail = 0
    for k, (wl, it, (J, b), inf, st) in enumerate(zip(wls, items, host, infos, stats)):
        if k == bad:
            continue
        if need[k] <= cap and st == 0:
            Jm = J if J is not None else np.zeros((0, wl.N))
            rr = gn.true_relres(wl.shape, wl.beta, Jm, wl.alpha, b, it["x"].cpu().numpy())
            assert rr <= 1.01e-8, (k, rr)
            n_ok += 1
        elif need[k] > cap:
            assert st == nat.H1W_ENOCONV, (k, st, need[k], cap)
            n_fail += 1
    print(f"maxit {cap}: {n_ok} instances solved, {n_fail} ENOCONV, instance {bad} ENUMERIC", flush=True)
    assert n_ok > 0 and n_fail > 0


def test_grouped_batch_solves_larger_items_one_at_a_time(P):
    # items with more than 128 rows do not fit a group's capacitance tile:
    # the grouped call solves them after the groups, one solve per item
    from paper_2209_02815_amd import _native as nat
    wls = H.batch_workloads(count=2, batch_id=12, sides=(17,), m_lo=129, m_hi=140) + \
        H.batch_workloads(count=2, batch_id=13, sides=(17,), m_lo=5, m_hi=10)
    items, host = make_items(wls)
    infos, stats, rep = nat.h1w_batch_solve(items, nworkers=2, rtol=1e-10, grouped=True)
    assert all(s == 0 for s in stats)
    for wl, it, (J, b), inf in zip(wls, items, host, infos):
        rr = gn.true_relres(wl.shape, wl.beta, J, wl.alpha, b, it["x"].cpu().numpy())
        assert rr <= 1.01e-10, (wl.name, rr)
        assert inf.iters > 0


def test_batch_bad_item_fails_alone(P):
    from paper_2209_02815_amd import _native as nat
    wls = small_batch()[:4]
    items, host = make_items(wls)
    items[2]["alpha"] = -1.0
    infos, stats, _ = nat.h1w_batch_solve(items, nworkers=2, rtol=1e-10, raise_on_error=False)
    assert stats[2] == nat.H1W_EINVAL
    assert [s for k, s in enumerate(stats) if k != 2] == [0, 0, 0]
    with pytest.raises(P.H1WError) as e:
        nat.h1w_batch_solve(items, nworkers=2, rtol=1e-10)
    assert e.value.status == nat.H1W_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replayed_vcycles_give_identical_solves(P, prec):
    # the V-cycles of the CG replayed from HIP graphs: every solve of a
    # sequence (different right-hand sides, row counts and grids, eager work
    # and synchronisations in between) is bitwise the eager solve
    rng = np.random.default_rng(9)
    for shape, ms in (((65, 65), (24, 40, 24)), ((17, 17, 17), (12, 30))):
        wl = H.workload("square129").with_(shape=shape, wid=900 + shape[0])
        with P.Context(shape, 1e-2, precision=prec) as ce, P.Context(shape, 1e-2, precision=prec, graphs=True) as cg:
            for m in ms:
                J = dev(H.j_rows(wl.with_(m=m)))
                b = dev(rng.standard_normal(wl.N))
                xe, ie = ce.gn_solve(J, 1e-4, b=b, rtol=1e-8 if prec == "mixed" else 1e-10)
                torch.cuda.synchronize()
                _ = (b * 2.0).sum().item()              # eager work between the solves
                xg, ig = cg.gn_solve(J, 1e-4, b=b, rtol=1e-8 if prec == "mixed" else 1e-10)
                torch.cuda.synchronize()
                assert ig.iters == ie.iters
                assert torch.equal(xg, xe), (shape, m)


def test_batch_with_graphs_matches_eager(P):
    from paper_2209_02815_amd import _native as nat
    wls = small_batch()
    items_e, host = make_items(wls)
    items_g, _ = make_items(wls)
    nat.h1w_batch_solve(items_e, nworkers=3, rtol=1e-10)
    infos, stats, _ = nat.h1w_batch_solve(items_g, nworkers=3, rtol=1e-10, graphs=True)
    assert all(s == 0 for s in stats)
    for a, b in zip(items_e, items_g):
        assert torch.equal(a["x"], b["x"])


def test_batch_workers_reused_across_batches(P):
    # The executor keeps its workers' contexts for the process: a second batch
    # on the same grids with another beta gets contexts of its own, an item
    # that fails inside its solve (a NaN right-hand side) does not leave a
    # broken context behind, and every solve is still right against the oracle.
    from paper_2209_02815_amd import _native as nat
    wls = H.batch_workloads(count=6, batch_id=8, sides=(17, 33), m_lo=4, m_hi=24)
    for beta in (1e-2, 3e-2, 1e-2):
        ws = [wl.with_(beta=beta) for wl in wls]
        items, host = make_items(ws)
        nanb = items[0]["b"].clone()
        nanb[3] = float("nan")
        bad = dict(items[0], b=nanb, x=torch.zeros_like(items[0]["x"]))
        infos, stats, _ = nat.h1w_batch_solve(items + [bad], precision=nat.H1W_FP64, nworkers=2, rtol=1e-10,
                                              raise_on_error=False)
        assert stats[-1] == nat.H1W_ENUMERIC and all(s == 0 for s in stats[:-1]), stats
        for wl, it, (J, b) in zip(ws, items, host):
            rr = gn.true_relres(wl.shape, wl.beta, J, wl.alpha, b, it["x"].cpu().numpy())
            assert rr <= 1.01e-10, (wl.name, beta, rr)


@pytest.mark.parametrize("prec,grouped", [("fp64", False), ("mixed", False), ("fp64", True), ("mixed", True)])
def test_full_batch_workload(P, prec, grouped):
    # the benchmark's batch at its real size: 256 2D instances, sides drawn
    # from {65, 129, 193, 257}, m in [16, 128], alpha log-uniform in
    # [1e-5, 1e-2], in the launch configurations bench.py times (one solve
    # per instance on 8 workers, or the grouped mode with one worker per
    # grid; autotuned); every instance's FP64 true residual recomputed by the
    # oracle
    from paper_2209_02815_amd import _native as nat
    rtol = 1e-8
    wls = H.batch_workloads()
    items, host = make_items(wls)
    precision = nat.H1W_FP64 if prec == "fp64" else nat.H1W_MIXED
    infos, stats, rep = nat.h1w_batch_solve(items, precision=precision, nworkers=8, autotune=1, rtol=rtol,
                                            grouped=grouped)
    assert all(s == 0 for s in stats) and rep.nworkers == (4 if grouped else 8)
    worst = 0.0
    for wl, it, (J, b), info in zip(wls, items, host, infos):
        x = it["x"].cpu().numpy()
        rr = gn.true_relres(wl.shape, wl.beta, J, wl.alpha, b, x)
        assert rr <= 1.01 * rtol, (wl.name, rr, info.as_dict())
        floor = gn.residual_rounding_floor(wl.shape, wl.beta, J, wl.alpha, b, x)
        assert abs(rr - info.relres_true) <= 1e-3 * rtol + floor, (wl.name, rr, info.relres_true, floor)
        worst = max(worst, rr)
    print(f"batch {prec} grouped={grouped}: 256 instances, worst oracle relres {worst:.2e}, "
          f"{sum(i.iters for i in infos)} iterations in total")
