#!/usr/bin/env python3
"""Benchmark: GMRES-GMG slab solves on one MI355X.

A step is one slab of the time marching on the 2D 256x256 workload (Q2/Q2/Q1,
dG(2), 7 levels from 4x4, vertex patches, tau = 1e-3), run inside the library
(stgmg_march): the right-hand side of Problem 3.1 from the previous slab's end
value on the device, then FGMRES(30) preconditioned by one V-cycle per
iteration, from x0 = 0 to a relative residual of 1e-8.
The hierarchy (level operators, patch inverses) is built once before timing
and stays resident in HBM; its setup time is reported separately.

Prints one JSON line.  Only the `cpu_baseline` leg imports the CPU oracle.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PATCH_KERNEL = {0: 'patch_apply_kernel', 1: 'patch_apply_tb_kernel', 2: 'patch_apply_red_kernel',
                3: 'patch_apply_red_sym_kernel (symmetric tiles)'}
# FP32 storage takes the tiles up to 96 Schur rows and the square layout beyond
PATCH_KERNEL_FP32_SYM = 'patch_apply_red_sym_kernel (FP32 paired tiles; patch_apply_red_kernel above 96 Schur rows)'
PATCH_SOLVE = {'full': 0, 'tb': 1, 'reduced': 2, 'sym': 3}
METRIC = "GMRES-GMG solves/s and V-cycle DoF/s at 1e-8 rel. residual; p50/p99 latency"


def kernel_source_hash():
    """sha256 prefix of the code of kernels.hip: comments (from // to the end of the line) and
    blank lines dropped, so that a counter record stays tied to the code it was measured on
    through edits of comments alone (the file holds no // inside string literals)."""
    import hashlib
    code = []
    with open(os.path.join(ROOT, 'paper_2303_06742_amd', 'csrc', 'kernels.hip')) as f:
        for line in f:
            c = line.split('//', 1)[0].rstrip()
            if c:
                code.append(c)
    return hashlib.sha256('\n'.join(code).encode()).hexdigest()[:16]


def measured_traffic(workload, precision, role='patch'):
    """HBM bytes per launch of the finest-level patch kernel (role 'patch') or operator kernel
    (role 'operator') from the rocprofv3 counter runs recorded in profiles/hbm_traffic.json, if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, 'profiles', 'hbm_traffic.json')
    if not os.path.exists(path):
        return None
    with open(path) as f:
        entries = json.load(f).get('entries', [])
    h = kernel_source_hash()
    for e in entries:
        if (e.get('workload') == workload and e.get('precision') == precision and e.get('kernels_hip_sha256') == h
                and e.get('role', 'patch') == role):
            return e['bytes_per_launch']
    return None


def measured_read_peak(torch):
    """Reference HBM read rate on this GPU: the best of torch.sum over a 4 GiB FP64 tensor and
    torch's device copy of the same (read + write counted), three timed runs each."""
    a = torch.ones(1 << 29, dtype=torch.float64, device='cuda')
    b = torch.empty_like(a)
    best = {}
    for name, fn, nbytes in (('sum', lambda: a.sum(), a.numel() * 8),
                              ('copy', lambda: b.copy_(a), 2 * a.numel() * 8)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            fn()
        e1.record()
        torch.cuda.synchronize()
        best[name] = nbytes / (e0.elapsed_time(e1) / 3 * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return best


def dense_inverse_bytes(cfg, w=8):
    """Bytes one finest-level sweep would move with the paper's dense patch inverses (Def:VankaOP
    literally): w * sum over patches of n_P^2 + 32 n.  Patch sizes by closed form: per axis a
    vertex patch spans 2 cells inside and 1 at the two boundary vertices, a cell patch 1."""
    from itertools import product
    from math import comb
    d, r, k, N = cfg.dim, cfg.r, cfg.k, cfg.fine_cells
    widths = [(2, N - 1), (1, 2)] if cfg.patch == 'vertex' else [(1, N)]
    nlp = comb(r - 1 + d, d)
    total = 0
    for combo in product(widths, repeat=d):
        mult, q, pp, cells = 1, 1, 1, 1
        for wdt, cnt in combo:
            mult *= cnt
            q *= r * wdt + 1
            pp *= (r - 1) * wdt + 1
            cells *= wdt
        if cfg.pressure == 'disc':
            pp = cells * nlp
        n_p = (k + 1) * (2 * d * q + pp)
        total += mult * n_p * n_p
    n1, n1p = r * N + 1, (r - 1) * N + 1
    n_s = 2 * d * n1 ** d + (N ** d * nlp if cfg.pressure == 'disc' else n1p ** d)
    return w * total + 32 * (k + 1) * n_s


def configs():
    from paper_2303_06742_amd import workloads as W
    return {'c2': W.C2, 'c1': W.C1, 'c3': W.C3, 'c3v': W.C3V, 'c2d': W.C2D}


def host_description():
    """CPU model, usable cores and RAM of the host the oracle runs on."""
    model, mem_gb = 'unknown', None
    try:
        with open('/proc/cpuinfo') as f:
            for line in f:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
        with open('/proc/meminfo') as f:
            for line in f:
                if line.startswith('MemTotal'):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {'cpu_model': model, 'cores_usable': len(os.sched_getaffinity(0)), 'nproc': os.cpu_count(),
            'ram_gb': mem_gb}


def cpu_baseline(cfg, sample_levels, n_full):
    """The oracle on one slab of the same physics on a smaller grid; solve time (setup excluded, as
    on the GPU) extrapolated linearly in unknowns.  Setup runs with a BLAS pool of every usable
    core; the solve is timed with one BLAS thread and with all cores, and the faster counts.
    Phases timed: assembly of the fine level, its patch extraction and inversion, the whole
    hierarchy, one V-cycle, the FGMRES solve."""
    from threadpoolctl import threadpool_limits
    from paper_2303_06742_amd import workloads as W
    from oracle import fgmres, gmg, problem
    scfg = W.scaled(cfg, sample_levels)
    host = host_description()
    cores = host['cores_usable']
    with threadpool_limits(limits=cores):
        Kc = scfg.K_cells()
        prm = problem.Params(rho=scfg.rho, lam=scfg.lam, mu=scfg.mu, alpha=scfg.alpha, c0=scfg.c0,
                             K=scfg.K if Kc is None else Kc, pressure=scfg.pressure, form=scfg.form)
        t0 = time.perf_counter()
        H = gmg.Hierarchy(scfg.dim, scfg.coarse_cells, scfg.levels - 1, scfg.r, scfg.k, scfg.tau, prm,
                          patch_kind=scfg.patch, J=scfg.n_smooth, omega=scfg.omega)
        t_setup = time.perf_counter() - t0
        # the fine level's two setup phases once more, separately (same calls the hierarchy makes)
        t0 = time.perf_counter()
        lev = gmg.Level(scfg.dim, scfg.fine_cells, scfg.r, scfg.k, scfg.tau, prm, scfg.patch)
        t_asm = time.perf_counter() - t0
        t0 = time.perf_counter()
        lev.build_smoother()
        t_inv = time.perf_counter() - t0
        del lev
        f = H.fine.prob
        sol = problem.ExactSolution(scfg.dim, *W.builtin_solution_exprs(scfg.dim), prm)
        F = problem.slab_rhs(f.blocks, scfg.k, scfg.tau, 0.0, problem.interpolate(f.blocks, sol, 0.0), sol)
    # the solve phase with one BLAS thread and with all cores: the oracle's small dense products
    # do not gain from a thread pool, so the faster of the two is the baseline
    runs = {}
    for nth in sorted({1, cores}):
        with threadpool_limits(limits=nth):
            t0 = time.perf_counter()
            H.precondition(F)
            t_vc = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, info = fgmres.fgmres(f.A, F, H.precondition, rtol=scfg.rtol, restart=scfg.restart)
            runs[nth] = (time.perf_counter() - t0, t_vc, info)
    best = min(runs, key=lambda t: runs[t][0])
    t_solve, t_vc, info = runs[best]
    blas_threads = best
    scale = n_full / f.n
    return {'value': 1.0 / (t_solve * scale), 'unit': 'solves/s', 'cores': blas_threads, 'kind': 'oracle',
            'sample': (f"one slab of the same physics on {scfg.fine_cells}^{scfg.dim} cells ({scfg.levels} levels, "
                       f"{f.n} unknowns, {info['iters']} FGMRES iterations): solve {t_solve:.2f} s, setup "
                       f"{t_setup:.2f} s; extrapolated linearly in unknowns (x{scale:.1f}) to the full grid; "
                       f"one Python process (NumPy/SciPy); solve timed with BLAS pools of 1 and {cores} threads, "
                       f"the faster ({blas_threads}) reported; setup with {cores}"),
            'solve_s_sample': t_solve,
            'phases_s': {'fine_assembly': t_asm, 'fine_patch_inversion': t_inv, 'hierarchy_setup': t_setup,
                         'vcycle': t_vc, 'solve': t_solve},
            'solve_s_by_blas_threads': {str(t): v[0] for t, v in runs.items()},
            'blas_threads': blas_threads, 'host': host}


def run_batch(args):
    """Independent 2D problems (16^2..128^2, dG(1)/dG(2), random physics, FP32 smoother, FP64 FGMRES),
    set up in waves that fit the HBM budget; each wave solved concurrently (stgmg_solve_batch) and,
    for comparison, one after another; then, with --compare-fp64, the same problems with FP64 patch
    solves one after another (the plain FP64 GPU solve), and the two solutions compared."""
    import numpy as np
    import torch
    from paper_2303_06742_amd import capi, workloads as W
    cfgs = W.batch_configs(args.batch_count, seed=args.seed)
    budget = int(args.hbm_budget_gb * 2 ** 30)
    t_setup = t_batch = t_seq = t_setup64 = t_seq64 = 0.0
    iters, iters64, res, max_dev, err64, fail64 = [], [], [], 0.0, [], []
    i = 0
    waves = 0
    while i < len(cfgs):
        wave, wcfg, used = [], [], 0
        while i < len(cfgs):
            _, res_b, peak_b = capi.footprint(cfgs[i], graph=args.graph)
            if wave and used + peak_b > budget:
                break
            t0 = time.perf_counter()
            wave.append(capi.Solver(cfgs[i], graph=args.graph))
            t_setup += time.perf_counter() - t0
            wcfg.append(cfgs[i])
            used += res_b
            i += 1
        waves += 1
        rhs = [torch.from_numpy(W.random_vector(s.n, 1000 + j)).cuda() for j, s in enumerate(wave)]
        xs = [s.empty() for s in wave]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = capi.solve_batch(wave, rhs, xs, rtol=1e-8)
        torch.cuda.synchronize()
        t_batch += time.perf_counter() - t0
        xq = [s.empty() for s in wave]
        t0 = time.perf_counter()
        for s, r, x in zip(wave, rhs, xq):
            s.solve(r, x, rtol=1e-8)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        for x, y, inf in zip(xs, xq, infos):
            max_dev = max(max_dev, float((x - y).abs().max()))
            iters.append(inf['iters'])
            res.append(inf['rel_res_true'])
        for s in wave:
            s.close()
        del xq
        if args.compare_fp64:
            # the plain FP64 GPU solve of the same problems, one problem at a time (set up, solve,
            # release: the FP64 hierarchies of a whole wave need more memory than the budget)
            for c64, r, x in zip(wcfg, rhs, xs):
                t0 = time.perf_counter()
                s64 = capi.Solver(c64, precision='fp64', graph=args.graph)
                torch.cuda.synchronize()
                t_setup64 += time.perf_counter() - t0
                y = s64.empty()
                t0 = time.perf_counter()
                try:
                    iters64.append(s64.solve(r, y, rtol=1e-8)['iters'])
                except capi.StgmgError as e:  # reported in the output line, not hidden
                    fail64.append({'problem': c64.name, 'error': str(e)})
                    print(f"[bench] FP64 comparison solve of {c64.name} failed: {e}", file=sys.stderr, flush=True)
                torch.cuda.synchronize()
                t_seq64 += time.perf_counter() - t0
                if not fail64 or fail64[-1]['problem'] != c64.name:
                    err64.append(float((x - y).abs().max() / y.abs().max()))
                s64.close()
                del y
        del xs, rhs
        torch.cuda.empty_cache()
        print(f"[bench] wave {waves}: {len(wave)} problems ({i}/{len(cfgs)})", file=sys.stderr, flush=True)
    n = len(cfgs)
    out = {'metric': 'batched GMRES-GMG solves/s (independent problems, 1e-8 rel. residual)', 'value': n / t_batch,
           'unit': 'solves/s', 'n_gpus': 1, 'steps': n, 'warmup': 0, 'ms_per_step': 1000 * t_batch / n,
           'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64+f32-smoother',
           'data': 'synthetic',
           'config': {'workload': f'batch of {n} 2D problems 16^2..128^2, dG(1)/dG(2), vertex patches, random '
                                  'physics, FP32 patch solves inside FP64 FGMRES',
                      'seed': args.seed, 'waves': waves, 'hbm_budget_gb': args.hbm_budget_gb, 'graph': args.graph},
           'sequential_solves_per_s': n / t_seq, 'setup_plus_solve_per_s': n / (t_setup + t_batch),
           'setup_s': t_setup, 'gmres_iters_mean': float(np.mean(iters)), 'rel_res_true_max': float(max(res)),
           'batch_vs_alone_max_abs_diff': max_dev}
    if args.compare_fp64:
        out['fp64_alone'] = {'solves_per_s': n / t_seq64, 'setup_plus_solve_per_s': n / (t_setup64 + t_seq64),
                             'setup_s': t_setup64, 'gmres_iters_mean': float(np.mean(iters64)),
                             'mixed_batched_over_fp64_alone': (n / t_batch) / (n / t_seq64),
                             'max_rel_err_mixed_vs_fp64': float(max(err64)) if err64 else None,
                             'failed_solves': fail64,
                             'note': 'the same problems and right-hand sides, FP64 patch solves, one problem at a time '
                                     '(solve time only in solves_per_s), same rtol 1e-8'}
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Serving loop: a seeded request mix (70% 2D 32^2..128^2 vertex patches, 30% 3D 8^3..16^3 cell
    patches, dG(1)/dG(2), half of them follow-on slabs of an earlier problem), first all at once
    (saturated throughput), then with Poisson arrivals at fractions of that throughput."""
    import numpy as np
    from paper_2303_06742_amd import capi, workloads as W
    mix = W.serve_mix(args.serve_count, seed=args.seed, sizes2d=tuple(args.serve_sizes_2d),
                      sizes3d=tuple(args.serve_sizes_3d))
    rhs = [W.random_vector(capi.footprint(cfg)[0], 2000 + j) for j, (_, cfg) in enumerate(mix)]
    budget = int(args.hbm_budget_gb * 2 ** 30)

    def run(rate, tag):
        srv = capi.Server(budget, max_slots=args.slots, resident_max=32)
        rng = np.random.default_rng(args.seed + 17)
        t0 = time.perf_counter()
        tickets = []
        for j, (key, cfg) in enumerate(mix):
            if rate:
                time.sleep(float(rng.exponential(1.0 / rate)))
            tickets.append(srv.submit(cfg, rhs[j], key=key + 1000 * hash(tag) % 1000000))
        lat, ok = [], 0
        for k, t in enumerate(tickets):
            # a request the server never finishes ends the run with an error instead of polling on
            st, _, inf, l = srv.wait(t, timeout_s=600.0)
            ok += int(st == capi.STGMG_OK and inf['converged'] == 1)
            lat.append(l)
            if (k + 1) % 40 == 0:
                print(f"[bench] serve {tag}: {k + 1}/{len(tickets)} done after {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
        el = time.perf_counter() - t0
        srv.close()
        print(f"[bench] serve {tag}: {len(mix) / el:.2f} solves/s p50 {np.percentile(lat, 50):.0f} ms", file=sys.stderr,
              flush=True)
        return {'offered_rate': rate, 'solves_per_s': len(mix) / el, 'p50_ms': float(np.percentile(lat, 50)),
                'p99_ms': float(np.percentile(lat, 99)), 'converged': ok}

    sat = run(0.0, 'saturated')
    rows = [run(f * sat['solves_per_s'], f'rate{f}') for f in args.serve_rates]
    out = {'metric': 'served GMRES-GMG solves/s with p50/p99 latency (setup on admission, resident reuse)',
           'value': sat['solves_per_s'], 'unit': 'solves/s', 'n_gpus': 1, 'steps': len(mix), 'warmup': 0,
           'ms_per_step': 1000.0 / sat['solves_per_s'], 'higher_is_better': True, 'scaling': 'weak',
           'vs_baseline': None, 'dtype': 'f64+f32-smoother', 'data': 'synthetic',
           'config': {'workload': f'{len(mix)} requests, 70% 2D {args.serve_sizes_2d}^2 vertex / 30% 3D '
                                  f'{args.serve_sizes_3d}^3 cell patches, dG(1)/dG(2), half follow-on slabs',
                      'seed': args.seed, 'slots': args.slots,
                      'hbm_budget_gb': args.hbm_budget_gb},
           'latency_ms_p50': sat['p50_ms'], 'latency_ms_p99': sat['p99_ms'], 'poisson': rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--config', default='c2', choices=['c2', 'c1', 'c3', 'c3v', 'c2d', 'batch', 'serve'])
    ap.add_argument('--batch-count', type=int, default=64)
    ap.add_argument('--serve-count', type=int, default=48)
    ap.add_argument('--serve-rates', type=float, nargs='*', default=[0.25, 0.5, 0.75, 0.9, 1.0, 1.25])
    ap.add_argument('--serve-sizes-2d', type=int, nargs='*', default=[32, 64, 128, 256])
    ap.add_argument('--serve-sizes-3d', type=int, nargs='*', default=[8, 16, 32])
    ap.add_argument('--compare-fp64', action='store_true',
                    help='batch: also solve every problem with FP64 patch solves, one after another')
    ap.add_argument('--slots', type=int, default=8)
    ap.add_argument('--seed', type=int, default=0)
    ap.add_argument('--hbm-budget-gb', type=float, default=200.0)
    ap.add_argument('--precision', default='fp64', choices=['fp64', 'fp32', 'bf16'])
    ap.add_argument('--form', default='v', choices=['v', 'dtu'],
                    help="third equation: 'v' Problem 3.1, 'dtu' Problem B.1")
    ap.add_argument('--graph', type=int, default=-1, choices=[-1, 0, 1],
                    help='V-cycle as a captured HIP graph: 1 captures it; 0 and -1 (automatic) launch directly')
    ap.add_argument('--waves', type=int, default=0, choices=[0, 1, 2, 4],
                    help='waves per patch of the tiled patch kernel: 0 by patch count or autotuned, 1, 2 or 4')
    ap.add_argument('--autotune', type=int, default=1, choices=[0, 1],
                    help='time the launch shapes of the patch and operator kernels at setup (default 1)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-sample-levels', type=int, default=None,
                    help='levels of the grid the oracle times (default: 32^2 cells in 2D, 8^3 in 3D)')
    ap.add_argument('--patch-solve', choices=sorted(PATCH_SOLVE), default=None,
                    help='storage of the patch solves: full space-time inverses, time blocks, or time blocks '
                         'with the u-equation rows eliminated (default: the workload default)')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='run a plain 1 GiB device copy first (reference for HBM byte counters)')
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (independent problems "
              "would be placed one per GPU; one large problem would be split into slabs of cells with "
              "halo exchanges).", file=sys.stderr)
        sys.exit(2)
    if args.config == 'batch':
        return run_batch(args)
    if args.config == 'serve':
        return run_serve(args)
    import numpy as np
    import torch
    from paper_2303_06742_amd import capi
    cfg = configs()[args.config]
    if args.patch_solve is not None:
        from paper_2303_06742_amd import workloads as W
        cfg = W.scaled(cfg, cfg.levels, name=cfg.name, time_blocks=PATCH_SOLVE[args.patch_solve])
    if args.form == 'dtu':  # Problem B.1 on the same workload
        from paper_2303_06742_amd import workloads as W
        cfg = W.scaled(cfg, cfg.levels, name=cfg.name + '-b1', form='dtu')
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # kernels of known traffic for the HBM counter runs: 1 GiB read + 1 GiB written by the
        # runtime's copy and by an elementwise kernel, 1 GiB read by a reduction
        a = torch.ones(1 << 27, dtype=torch.float64, device='cuda')
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
            torch.mul(a, 1.0, out=b)
            a.sum()
        torch.cuda.synchronize()
        del a, b
    print(f"[bench] setup {cfg.name} {args.precision}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    S = capi.Solver(cfg, precision=args.precision, graph=args.graph, waves=args.waves, autotune=args.autotune)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    q = S.query(-1)
    k, ns, n = cfg.k, S.ns, S.n
    state = {'t': 0.0, 'Xend': S.interpolate_solution(0.0)}
    x = S.empty()
    kept = []  # mixed precision: (t, start values, x) of every timed slab, compared with FP64 afterwards

    def step(keep=False):
        # one slab inside the library (stgmg_march): right-hand side on the device from the end
        # values of the previous slab (updated in place), x0 = 0, FGMRES-GMG to rtol
        start = state['Xend'].clone() if keep else None
        _, infos_ = S.march(state['t'], 1, state['Xend'], x, rtol=cfg.rtol, restart=cfg.restart)
        if keep:
            kept.append((state['t'], start, x.clone()))
        state['t'] += cfg.tau
        return infos_[0]

    print(f"[bench] setup {setup_s:.1f} s, n={n}; warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    S.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        infos.append(step(keep=args.precision != 'fp64'))
        print(f"[bench] step {i}: {infos[-1]['iters']} its, {infos[-1]['t_solve_ms']:.1f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pa = S.profile_get(capi.PROF_PATCH_APPLY)
    rs = S.profile_get(capi.PROF_RESIDUAL)
    S.profile(False)
    exact = S.interpolate_solution(state['t'])
    nodal_err = float((state['Xend'] - exact).abs().max() / exact.abs().max())
    iters = [i['iters'] for i in infos]
    lat = np.array([i['t_solve_ms'] for i in infos])
    ms_per_step = 1000.0 * elapsed / args.steps
    avg_pa_ms = pa['total_ms'] / max(pa['launches'], 1)
    achieved = pa['bytes_per_launch'] / (avg_pa_ms * 1e-3) / 1e9 if pa['launches'] else 0.0
    avg_rs_ms = rs['total_ms'] / max(rs['launches'], 1)
    out = {
        'metric': METRIC,
        'value': args.steps / elapsed,
        'unit': 'solves/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': ms_per_step,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f64' if args.precision == 'fp64' else f'f64+{"f32" if args.precision == "fp32" else "bf16"}-smoother',
        'data': 'synthetic',
        'config': {'workload': cfg.name, 'dim': cfg.dim, 'cells': f"{cfg.fine_cells}^{cfg.dim}",
                   'levels': cfg.levels, 'r': cfg.r, 'k': cfg.k, 'patch': cfg.patch, 'pressure': cfg.pressure, 'form': cfg.form, 'smoother': args.precision,
                   'tau': cfg.tau, 'unknowns': n, 'nnz': q['nnz'], 'patches': q['patches'], 'rtol': cfg.rtol,
                   'restart': cfg.restart, 'waves_per_patch': args.waves, 'autotune': args.autotune},
        'vcycle_dof_per_s': n * sum(iters) / elapsed,
        'latency_ms_p50': float(np.percentile(lat, 50)),
        'latency_ms_p99': float(np.percentile(lat, 99)),
        'gmres_iters': iters,
        'rel_res_true_max': max(i['rel_res_true'] for i in infos),
        'nodal_err_vs_exact': nodal_err,
        'setup_s': setup_s,
        'launch_shapes': [dict(level=l, **S.query_launch(l)) for l in range(S.levels)],
        'hbm_bytes_resident': q['bytes'],
        'roofline': {'bound': 'hbm', 'kernel': (PATCH_KERNEL_FP32_SYM if args.precision == 'fp32' and cfg.time_blocks == 3
                                                else PATCH_KERNEL[3] + ' BF16' if args.precision == 'bf16'
                                                else PATCH_KERNEL[cfg.time_blocks]) + ' (finest level)',
                     'achieved': achieved,
                     'peak': HBM_PEAK_GBS, 'unit': 'GB/s', 'frac': achieved / HBM_PEAK_GBS,
                     'traffic': measured_traffic(cfg.name, args.precision), 'kernels_hip_sha256': kernel_source_hash(),
                     'avg_launch_ms': avg_pa_ms, 'launches': pa['launches'],
                     'bytes_per_launch': pa['bytes_per_launch'],
                     # context: the same sweep with the paper's dense A_P^{-1} (the per-unit figure
                     # w * sum n_P^2 + 32 n) would have to move this many bytes; the rate is the
                     # equivalent throughput of the reformulated patch solve, not HBM traffic
                     'dense_inverse_equivalent': {
                         'bytes_per_launch': dense_inverse_bytes(cfg, {'fp64': 8, 'fp32': 4, 'bf16': 2}[args.precision]),
                         'GBs': dense_inverse_bytes(cfg, {'fp64': 8, 'fp32': 4, 'bf16': 2}[args.precision]) /
                         (avg_pa_ms * 1e-3) / 1e9 if pa['launches'] else 0.0}},
        'residual_spmv': {'kernel': 'node_op_kernel (finest level)', 'avg_launch_ms': avg_rs_ms,
                          'launches': rs['launches'], 'bytes_per_launch': rs['bytes_per_launch'],
                          'achieved_GBs': rs['bytes_per_launch'] / (avg_rs_ms * 1e-3) / 1e9 if rs['launches'] else 0,
                          'traffic': measured_traffic(cfg.name, args.precision, 'operator')},
    }
    S.close()
    if kept:
        # per result: the mixed-precision solution and the plain FP64 path's solution of the same
        # slab system, both at the workload's rtol, against an FP64 solve of that system to 1e-12
        # (the FP64 path agrees with the oracle to 1e-10 in the parity tests): equal final
        # accuracy shows as errors of the same size
        S64 = capi.Solver(cfg, precision='fp64', graph=args.graph)
        errs, errs64, iters64 = [], [], []
        for t_, start_, x_ in kept:
            r_ = S64.slab_rhs(t_, start_)
            x64, xref = S64.empty(), S64.empty()
            i64 = S64.solve(r_, x64, rtol=cfg.rtol, restart=cfg.restart)
            S64.solve(r_, xref, rtol=1e-12, restart=cfg.restart, max_iters=200)
            iters64.append(i64['iters'])
            nrm = xref.abs().max()
            errs.append(float((x_ - xref).abs().max() / nrm))
            errs64.append(float((x64 - xref).abs().max() / nrm))
        S64.close()
        out['mixed_vs_fp64'] = {'max_rel_err_per_result': errs, 'max_rel_err': max(errs),
                                'fp64_max_rel_err_per_result': errs64, 'fp64_max_rel_err': max(errs64),
                                'fp64_gmres_iters': iters64,
                                'reference': 'FP64 GPU solve of the same slab right-hand side to rtol 1e-12; '
                                             'max_rel_err: the mixed-precision solution at the workload rtol, '
                                             'fp64_max_rel_err: the plain FP64 solution at the same rtol'}
        del kept[:]
    if not args.copy_calibration:  # counter runs keep to the calibration kernels' known sizes
        peak = measured_read_peak(torch)
        # torch's own streaming kernels on the same GPU, for context (not the roofline peak)
        out['roofline']['torch_stream_reference'] = {'unit': 'GB/s', 'sum': peak['sum'], 'copy': peak['copy'],
                                                     'achieved_over_best': achieved / max(peak.values())}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        lv = args.cpu_sample_levels or (4 if cfg.dim == 2 else 2)
        out['cpu_baseline'] = cpu_baseline(cfg, min(lv, cfg.levels), n)
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
