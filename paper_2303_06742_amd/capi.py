"""ctypes binding of the C ABI in include/stgmg.h (argument marshalling only).

Every computation happens in libstgmg.so (HIP kernels for gfx950).  Device
vectors are torch tensors on a ROCm device, float64 and contiguous; torch is
used for device memory and the stream handle only.  If the library is missing
this module raises at import: there is no fallback path.
"""
import ctypes
import os

import numpy as np
# torch brings its own HIP and HSA runtime libraries.  It is loaded before libstgmg.so so that the
# process holds the runtime torch uses when the library is loaded: with the library loaded first, a
# process that then initialised torch found no device in the library's HIP calls.
import torch  # noqa: F401  (device memory and streams)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libstgmg.so')

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

STGMG_OK = 0
STGMG_NOT_CONVERGED = 1
STGMG_PENDING = 2
STGMG_ERR_INVALID_ARG = -1
STGMG_ERR_UNSUPPORTED = -2
STGMG_ERR_OOM = -3
STGMG_ERR_HIP = -4
STGMG_ERR_SINGULAR_PATCH = -5
STGMG_ERR_NONFINITE = -6
STGMG_ERR_BAD_POINTER = -7
PATCH = {'cell': 0, 'vertex': 1}
PROF_PATCH_APPLY = 0
PROF_RESIDUAL = 1
PREC = {'fp64': 0, 'fp32': 1, 'bf16': 2}
PRESSURE = {'cont': 0, 'disc': 1}  # Q_{r-1} (Taylor-Hood) or P_{r-1}^disc with the interior penalty form
FORM = {'v': 0, 'dtu': 1}  # Problem 3.1 or Problem B.1


class Params(ctypes.Structure):
    _fields_ = [('dim', ctypes.c_int32), ('coarse_cells', ctypes.c_int32), ('levels', ctypes.c_int32),
                ('r', ctypes.c_int32), ('k', ctypes.c_int32), ('patch', ctypes.c_int32),
                ('smoother_prec', ctypes.c_int32), ('n_smooth', ctypes.c_int32), ('omega', ctypes.c_double),
                ('tau', ctypes.c_double), ('rho', ctypes.c_double), ('lam', ctypes.c_double),
                ('mu', ctypes.c_double), ('alpha', ctypes.c_double), ('c0', ctypes.c_double),
                ('K', ctypes.c_double), ('K_cells', ctypes.c_void_p), ('graph', ctypes.c_int32),
                ('time_blocks', ctypes.c_int32), ('pressure', ctypes.c_int32), ('form', ctypes.c_int32),
                ('waves_per_patch', ctypes.c_int32), ('autotune', ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [('iters', ctypes.c_int32), ('restarts', ctypes.c_int32), ('converged', ctypes.c_int32),
                ('res0', ctypes.c_double), ('rel_res_true', ctypes.c_double), ('rel_res_est', ctypes.c_double),
                ('t_solve_ms', ctypes.c_double), ('t_vcycle_ms', ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


_H = ctypes.c_void_p
_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_S = ctypes.c_int32


def _decl(name, args, res=_S):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


stgmg_setup = _decl('stgmg_setup', [ctypes.POINTER(Params), _P, ctypes.POINTER(_H)])
stgmg_query = _decl('stgmg_query', [_H, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                    ctypes.POINTER(_I64)])
stgmg_query_launch = _decl('stgmg_query_launch', [_H, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)])
stgmg_solve = _decl('stgmg_solve', [_H, _P, _P, _D, _I32, _I32, ctypes.POINTER(Info)])
stgmg_solve_noalloc = _decl('stgmg_solve_noalloc', [_H, _P, _P, _D, _I32, _I32, ctypes.POINTER(Info)])
stgmg_apply_operator = _decl('stgmg_apply_operator', [_H, _I32, _P, _P])
stgmg_apply_vcycle = _decl('stgmg_apply_vcycle', [_H, _P, _P])
stgmg_smooth = _decl('stgmg_smooth', [_H, _I32, _P, _P, _I32])
stgmg_prolongate_add = _decl('stgmg_prolongate_add', [_H, _I32, _P, _P])
stgmg_restrict = _decl('stgmg_restrict', [_H, _I32, _P, _P])
stgmg_slab_rhs = _decl('stgmg_slab_rhs', [_H, _D, _P, _P])
stgmg_march = _decl('stgmg_march', [_H, _D, _I32, _P, _P, _D, _I32, _I32, ctypes.POINTER(Info)])
stgmg_interpolate_solution = _decl('stgmg_interpolate_solution', [_H, _D, _P])
stgmg_get_patch_inverse = _decl('stgmg_get_patch_inverse', [_H, _I32, _I64, ctypes.POINTER(_I32), _P, _P])
stgmg_profile_enable = _decl('stgmg_profile_enable', [_H, _I32])
stgmg_profile_get = _decl('stgmg_profile_get', [_H, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_D),
                                                ctypes.POINTER(_D)])
stgmg_footprint = _decl('stgmg_footprint', [ctypes.POINTER(Params), _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                            ctypes.POINTER(_I64)])
stgmg_solve_batch = _decl('stgmg_solve_batch', [_I32, ctypes.POINTER(_H), ctypes.POINTER(_P), ctypes.POINTER(_P), _D,
                                                _I32, _I32, ctypes.POINTER(Info), ctypes.POINTER(_S)])
stgmg_server_create = _decl('stgmg_server_create', [_I64, _I32, _I32, ctypes.POINTER(_P)])
stgmg_server_submit = _decl('stgmg_server_submit', [_P, ctypes.POINTER(Params), ctypes.c_uint64, _P, _D,
                                                    ctypes.POINTER(ctypes.c_uint64)])
stgmg_server_poll = _decl('stgmg_server_poll', [_P, ctypes.c_uint64, _P, ctypes.POINTER(Info), ctypes.POINTER(_D)])
stgmg_server_destroy = _decl('stgmg_server_destroy', [_P])
stgmg_server_message = _decl('stgmg_server_message', [_P, ctypes.c_uint64], ctypes.c_char_p)
stgmg_destroy = _decl('stgmg_destroy', [_H])
stgmg_status_string = _decl('stgmg_status_string', [_S], ctypes.c_char_p)
stgmg_last_error = _decl('stgmg_last_error', [], ctypes.c_char_p)

EXPORTED = ['stgmg_setup', 'stgmg_query', 'stgmg_query_launch', 'stgmg_solve', 'stgmg_solve_noalloc', 'stgmg_apply_operator', 'stgmg_apply_vcycle',
            'stgmg_smooth', 'stgmg_prolongate_add', 'stgmg_restrict', 'stgmg_slab_rhs', 'stgmg_march',
            'stgmg_interpolate_solution', 'stgmg_get_patch_inverse', 'stgmg_profile_enable', 'stgmg_profile_get',
            'stgmg_destroy', 'stgmg_status_string', 'stgmg_last_error', 'stgmg_footprint', 'stgmg_solve_batch',
            'stgmg_server_create', 'stgmg_server_submit', 'stgmg_server_poll', 'stgmg_server_message',
            'stgmg_server_destroy']


class StgmgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = stgmg_last_error().decode(errors='replace')
        super().__init__(f"{where}: {stgmg_status_string(status).decode()} ({status}): {msg}")


def check(status, where, allow=(STGMG_OK,)):
    if status not in allow:
        raise StgmgError(status, where)
    return status


def _dptr(t, n=None):
    """Device pointer of a contiguous float64 tensor on a ROCm device, with a size check."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def make_params(cfg, precision=None, graph=-1, time_blocks=None, waves=0, autotune=0):
    """(Params, K array kept alive by the caller) for a workloads.Config.  waves: waves per patch of
    the tiled patch solve (0 by patch count, 1 or 4); autotune: 1 to time the launch shapes at setup."""
    K = cfg.K_cells()
    if K is not None:
        K = np.ascontiguousarray(K, dtype=np.float64)
    p = Params(dim=cfg.dim, coarse_cells=cfg.coarse_cells, levels=cfg.levels, r=cfg.r, k=cfg.k,
               patch=PATCH[cfg.patch], smoother_prec=PREC[precision or cfg.precision], n_smooth=cfg.n_smooth,
               omega=cfg.omega, tau=cfg.tau, rho=cfg.rho, lam=cfg.lam, mu=cfg.mu, alpha=cfg.alpha, c0=cfg.c0,
               K=cfg.K, K_cells=None if K is None else K.ctypes.data, graph=graph,
               time_blocks=cfg.time_blocks if time_blocks is None else time_blocks,
               pressure=PRESSURE[cfg.pressure], form=FORM[cfg.form], waves_per_patch=waves, autotune=autotune)
    return p, K


def footprint(cfg, precision=None, restart=30, graph=-1, time_blocks=None):
    """Closed-form (n, resident bytes, setup peak bytes) without building anything."""
    p, _K = make_params(cfg, precision, graph, time_blocks)
    n, res, peak = _I64(), _I64(), _I64()
    check(stgmg_footprint(ctypes.byref(p), restart, ctypes.byref(n), ctypes.byref(res), ctypes.byref(peak)),
          'stgmg_footprint')
    return n.value, res.value, peak.value


def solve_batch(solvers, rhs, xs, rtol=1e-8, restart=30, max_iters=1000):
    """Solve independent problems at once (stgmg_solve_batch); returns per-problem info dicts."""
    cnt = len(solvers)
    hs = (_H * cnt)(*[s.h for s in solvers])
    rp = (_P * cnt)(*[_dptr(r, s.n).value for r, s in zip(rhs, solvers)])
    xp = (_P * cnt)(*[_dptr(x, s.n).value for x, s in zip(xs, solvers)])
    infos = (Info * cnt)()
    sts = (_S * cnt)()
    stgmg_solve_batch(cnt, hs, rp, xp, rtol, restart, max_iters, infos, sts)
    for i in range(cnt):
        check(sts[i], f'stgmg_solve_batch[{i}]', allow=(STGMG_OK, STGMG_NOT_CONVERGED))
    return [infos[i].as_dict() for i in range(cnt)]


class Server:
    """The serving loop (stgmg_server_*): host vectors in, host vectors out."""

    def __init__(self, hbm_budget, max_slots=8, resident_max=16):
        s = _P()
        check(stgmg_server_create(hbm_budget, max_slots, resident_max, ctypes.byref(s)), 'stgmg_server_create')
        self.s = s
        self.n = {}

    def submit(self, cfg, rhs, key=0, rtol=1e-8, precision=None):
        p, _K = make_params(cfg, precision)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        t = ctypes.c_uint64()
        check(stgmg_server_submit(self.s, ctypes.byref(p), key, rhs.ctypes.data_as(_P), rtol, ctypes.byref(t)),
              'stgmg_server_submit')
        self.n[t.value] = rhs.shape[0]
        return t.value

    def poll(self, ticket):
        """None while pending, else (status, x, info, latency_ms)."""
        x = np.empty(self.n[ticket])
        info = Info()
        lat = _D()
        st = stgmg_server_poll(self.s, ticket, x.ctypes.data_as(_P), ctypes.byref(info), ctypes.byref(lat))
        if st == STGMG_PENDING:
            return None
        return st, x, info.as_dict(), lat.value

    def message(self, ticket):
        """Error text of a finished request that failed ('' otherwise)."""
        return stgmg_server_message(self.s, ticket).decode(errors='replace')

    def wait(self, ticket, poll_s=0.0005, timeout_s=None):
        """Poll until the request is done; TimeoutError after timeout_s seconds (None: no limit)."""
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if timeout_s is not None and time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"server request {ticket} not done after {timeout_s} s")
            time.sleep(poll_s)

    def close(self):
        if getattr(self, 's', None):
            stgmg_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One problem hierarchy (stgmg_setup) and the calls on it."""

    def __init__(self, cfg, precision=None, stream=None, graph=-1, time_blocks=None, waves=0, autotune=0):
        import torch
        self._torch = torch
        self.cfg = cfg
        p, self._K = make_params(cfg, precision, graph, time_blocks, waves, autotune)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _H()
        check(stgmg_setup(ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), 'stgmg_setup')
        self.h = h
        self.levels = cfg.levels
        self.n = self.query(-1)['n']
        self.ns = self.n // (cfg.k + 1)

    def query(self, level=-1):
        n, npch, nnz, b = _I64(), _I64(), _I64(), _I64()
        check(stgmg_query(self.h, level, ctypes.byref(n), ctypes.byref(npch), ctypes.byref(nnz), ctypes.byref(b)),
              'stgmg_query')
        return {'n': n.value, 'patches': npch.value, 'nnz': nnz.value, 'bytes': b.value}

    def query_launch(self, level=-1):
        w, g = _I32(), _I32()
        check(stgmg_query_launch(self.h, level, ctypes.byref(w), ctypes.byref(g)), 'stgmg_query_launch')
        return {'waves_per_patch': w.value, 'node_lanes': g.value}

    def empty(self, n=None):
        return self._torch.zeros(self.n if n is None else n, dtype=self._torch.float64, device='cuda')

    def solve(self, rhs, x, rtol=1e-8, restart=30, max_iters=1000):
        info = Info()
        st = stgmg_solve(self.h, _dptr(rhs, self.n), _dptr(x, self.n), rtol, restart, max_iters, ctypes.byref(info))
        check(st, 'stgmg_solve', allow=(STGMG_OK, STGMG_NOT_CONVERGED))
        return info.as_dict()

    def apply_operator(self, x, level=-1, y=None):
        n = self.query(level)['n']
        y = self.empty(n) if y is None else y
        check(stgmg_apply_operator(self.h, level, _dptr(x, n), _dptr(y, n)), 'stgmg_apply_operator')
        return y

    def vcycle(self, r, z=None):
        z = self.empty() if z is None else z
        check(stgmg_apply_vcycle(self.h, _dptr(r, self.n), _dptr(z, self.n)), 'stgmg_apply_vcycle')
        return z

    def smooth(self, level, b, d, sweeps):
        n = self.query(level)['n']
        check(stgmg_smooth(self.h, level, _dptr(b, n), _dptr(d, n), sweeps), 'stgmg_smooth')
        return d

    def prolongate_add(self, level, e, d):
        check(stgmg_prolongate_add(self.h, level, _dptr(e, self.query(level - 1)['n']),
                                   _dptr(d, self.query(level)['n'])), 'stgmg_prolongate_add')
        return d

    def restrict(self, level, r):
        b = self.empty(self.query(level - 1)['n'])
        check(stgmg_restrict(self.h, level, _dptr(r, self.query(level)['n']), _dptr(b)), 'stgmg_restrict')
        return b

    def slab_rhs(self, t_start, x_prev_end, rhs=None):
        rhs = self.empty() if rhs is None else rhs
        check(stgmg_slab_rhs(self.h, t_start, _dptr(x_prev_end, self.ns), _dptr(rhs, self.n)), 'stgmg_slab_rhs')
        return rhs

    def march(self, t_start, n_slabs, x_end, x=None, rtol=1e-8, restart=30, max_iters=1000):
        """stgmg_march: n_slabs slabs of time marching inside the library; x_end (n_s values) is
        updated in place to the end values; returns (x of the last slab, per-slab info dicts)."""
        x = self.empty() if x is None else x
        infos = (Info * max(n_slabs, 1))()
        st = stgmg_march(self.h, t_start, n_slabs, _dptr(x_end, self.ns), _dptr(x, self.n), rtol, restart, max_iters,
                         infos)
        check(st, 'stgmg_march', allow=(STGMG_OK, STGMG_NOT_CONVERGED))
        return x, [infos[i].as_dict() for i in range(n_slabs)]

    def interpolate_solution(self, t):
        out = self.empty(self.ns)
        check(stgmg_interpolate_solution(self.h, t, _dptr(out, self.ns)), 'stgmg_interpolate_solution')
        return out

    def patch_inverse(self, level, patch):
        npp = _I32()
        check(stgmg_get_patch_inverse(self.h, level, patch, ctypes.byref(npp), None, None), 'stgmg_get_patch_inverse')
        out = np.zeros((npp.value, npp.value))
        dofs = np.zeros(npp.value, dtype=np.int64)
        check(stgmg_get_patch_inverse(self.h, level, patch, ctypes.byref(npp), out.ctypes.data_as(_P),
                                      dofs.ctypes.data_as(_P)), 'stgmg_get_patch_inverse')
        return out, dofs

    def profile(self, enable):
        check(stgmg_profile_enable(self.h, 1 if enable else 0), 'stgmg_profile_enable')

    def profile_get(self, what):
        n, ms, b = _I64(), _D(), _D()
        check(stgmg_profile_get(self.h, what, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)), 'stgmg_profile_get')
        return {'launches': n.value, 'total_ms': ms.value, 'bytes_per_launch': b.value}

    def close(self):
        if getattr(self, 'h', None):
            stgmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
