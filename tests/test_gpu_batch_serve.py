"""Batched solves and the serving loop: footprints, and results that are the same
alone and in a mix (bitwise: no reduction crosses problems)."""
import numpy as np
import pytest

from tests.gpu_util import CONFIGS, oracle_direct_solve, require_gpu, to_dev, to_host
from paper_2303_06742_amd import workloads

pytestmark = pytest.mark.gpu


def capi():
    require_gpu()
    from paper_2303_06742_amd import capi as c
    return c


@pytest.mark.parametrize("key", ['c1', 'c2s', 'c3s', 'c2s_b1', 'c1_disc', 'c2d', 'c3s_disc_b1'])
def test_footprint_is_what_setup_allocates(key):
    c = capi()
    cfg = CONFIGS[key]
    n, res, peak = c.footprint(cfg)
    S = c.Solver(cfg)
    x = S.empty()
    S.solve(to_dev(workloads.random_vector(S.n, 1)), x)  # allocates the Krylov workspace
    q = S.query(-1)
    assert n == S.n and q['bytes'] == res and peak >= res
    S.close()


def test_batch_equals_alone():
    c = capi()
    cfgs = workloads.batch_configs(4, seed=3, sizes=(16, 32))
    solvers = [c.Solver(cfg) for cfg in cfgs]
    rhs = [to_dev(workloads.random_vector(s.n, 10 + i)) for i, s in enumerate(solvers)]
    alone = []
    for s, r in zip(solvers, rhs):
        x = s.empty()
        s.solve(r, x)
        alone.append(to_host(x))
    xs = [s.empty() for s in solvers]
    infos = c.solve_batch(solvers, rhs, xs)
    for a, x, i in zip(alone, xs, infos):
        assert i['converged'] == 1 and np.array_equal(a, to_host(x))
    for s in solvers:
        s.close()


def test_server_alone_and_in_mix():
    c = capi()
    target = workloads.batch_configs(1, seed=5, sizes=(32,))[0]
    n, _, _ = c.footprint(target)
    F = workloads.random_vector(n, 99)
    srv = c.Server(hbm_budget=64 << 30, max_slots=4, resident_max=4)
    st, x_alone, info, lat = srv.wait(srv.submit(target, F, key=1))
    assert st == c.STGMG_OK and info['converged'] == 1
    # the same request inside a mix of other problems, some of them resident follow-ons
    mix = workloads.serve_mix(8, seed=6, sizes2d=(16, 32), sizes3d=(4,))
    tickets = []
    for j, (key, cfg) in enumerate(mix):
        nn, _, _ = c.footprint(cfg)
        tickets.append(srv.submit(cfg, workloads.random_vector(nn, 200 + j), key=100 + key))
        if j == 3:
            t_target = srv.submit(target, F, key=1)  # resident hierarchy reused
    for t in tickets:
        st2, _, inf2, _ = srv.wait(t)
        assert st2 == c.STGMG_OK and inf2['converged'] == 1
    st, x_mix, info2, _ = srv.wait(t_target)
    assert st == c.STGMG_OK and np.array_equal(x_alone, x_mix)
    srv.close()


def test_server_every_result_same_alone_and_in_mix():
    """Twelve requests (repeated keys = follow-on slabs on resident hierarchies, evictions under a
    tight budget) run concurrently; each result equals the same request solved alone, bitwise."""
    c = capi()
    mix = workloads.serve_mix(12, seed=8, sizes2d=(16, 32), sizes3d=(4,))
    rhs = [workloads.random_vector(c.footprint(cfg)[0], 300 + j) for j, (_, cfg) in enumerate(mix)]
    alone = []
    solo = c.Server(hbm_budget=64 << 30, max_slots=1, resident_max=0)
    for (key, cfg), F in zip(mix, rhs):
        st, x, info, _ = solo.wait(solo.submit(cfg, F))
        assert st == c.STGMG_OK
        alone.append(x)
    solo.close()
    peak = max(c.footprint(cfg)[2] + 16 * len(F) for (_, cfg), F in zip(mix, rhs))
    srv = c.Server(hbm_budget=3 * peak, max_slots=4, resident_max=3)
    tickets = [srv.submit(cfg, F, key=key) for (key, cfg), F in zip(mix, rhs)]
    for t, x0 in zip(tickets, alone):
        st, x, info, _ = srv.wait(t)
        assert st == c.STGMG_OK and info['converged'] == 1 and np.array_equal(x, x0)
    srv.close()


def test_server_staggered_arrivals_all_succeed():
    """Requests that arrive while others run (setups overlapping other workers' uploads,
    solves and downloads) all finish OK and converged, with no error text, and equal the
    same requests solved one at a time.  (A hierarchy captured as a HIP graph in one worker
    once made the other workers' null-stream copies fail.)"""
    import time
    c = capi()
    mix = workloads.serve_mix(16, seed=12, sizes2d=(16, 32, 64), sizes3d=(4, 8))
    rhs = [workloads.random_vector(c.footprint(cfg)[0], 500 + j) for j, (_, cfg) in enumerate(mix)]
    solo = c.Server(hbm_budget=64 << 30, max_slots=1, resident_max=0)
    alone = []
    for (key, cfg), F in zip(mix, rhs):
        t0 = solo.submit(cfg, F)
        st, x, info, _ = solo.wait(t0)
        assert st == c.STGMG_OK, solo.message(t0)
        alone.append(x)
    solo.close()
    srv = c.Server(hbm_budget=64 << 30, max_slots=4, resident_max=8)
    rng = np.random.default_rng(13)
    tickets = []
    for (key, cfg), F in zip(mix, rhs):
        time.sleep(float(rng.exponential(0.01)))
        tickets.append(srv.submit(cfg, F, key=key))
    for j, (t, x0) in enumerate(zip(tickets, alone)):
        st, x, info, _ = srv.wait(t)
        assert st == c.STGMG_OK and info['converged'] == 1, (j, st, srv.message(t))
        assert srv.message(t) == ''
        assert np.array_equal(x, x0), j
    srv.close()


def test_server_refuses_what_cannot_fit():
    c = capi()
    cfg = CONFIGS['c2s']
    n, res, peak = c.footprint(cfg)
    srv = c.Server(hbm_budget=res // 2, max_slots=1, resident_max=0)
    with pytest.raises(c.StgmgError) as e:
        srv.submit(cfg, np.zeros(n))
    assert e.value.status == c.STGMG_ERR_OOM
    srv.close()


def _check_against_oracle(cfg, F, x, info, what):
    ref, A = oracle_direct_solve(cfg, F)
    res = np.linalg.norm(F - A @ x) / np.linalg.norm(F)
    err = np.abs(x - ref).max() / np.abs(ref).max()
    print(f"[{what}] {cfg.name} iters={info['iters']} rel_res={res:.2e} err_vs_oracle={err:.2e}", flush=True)
    assert info['converged'] == 1 and res <= 1e-10 * (1 + 1e-6) and err < 1e-7


def test_batch_against_oracle():
    """Batched random-physics problems (FP32 patch solves, FP64 FGMRES, rtol 1e-10) against the
    oracle's sparse direct solve of the same problems: residual through the oracle's operator
    <= 1e-10 and solution error < 1e-7."""
    c = capi()
    cfgs = workloads.batch_configs(3, seed=21, sizes=(16,))
    solvers = [c.Solver(cfg) for cfg in cfgs]
    F = [workloads.random_vector(s.n, 40 + i) for i, s in enumerate(solvers)]
    xs = [s.empty() for s in solvers]
    infos = c.solve_batch(solvers, [to_dev(f) for f in F], xs, rtol=1e-10)
    for cfg, f, x, info in zip(cfgs, F, xs, infos):
        _check_against_oracle(cfg, f, to_host(x), info, 'batch')
    for s in solvers:
        s.close()


def test_server_against_oracle():
    """Served random-physics requests (a 2D vertex-patch and a 3D cell-patch problem, FP32 patch
    solves) against the oracle's sparse direct solve, as in the batch test."""
    c = capi()
    mix = workloads.serve_mix(6, seed=31, sizes2d=(16,), sizes3d=(4,), p3d=0.5, p_follow=0.0)
    picked = [next(m for m in mix if m[1].dim == 2), next(m for m in mix if m[1].dim == 3)]
    srv = c.Server(hbm_budget=64 << 30, max_slots=2, resident_max=2)
    reqs = []
    for j, (key, cfg) in enumerate(picked):
        F = workloads.random_vector(c.footprint(cfg)[0], 70 + j)
        reqs.append((cfg, F, srv.submit(cfg, F, key=key, rtol=1e-10)))
    for cfg, F, t in reqs:
        st, x, info, _ = srv.wait(t)
        assert st == c.STGMG_OK, srv.message(t)
        _check_against_oracle(cfg, F, x, info, 'serve')
    srv.close()
