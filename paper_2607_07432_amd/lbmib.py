"""Python binding of the HIP library (include/lbmib.h): argument marshalling only.

PyTorch supplies the device workspace and the HIP stream; every step of the
method runs in the library's kernels. Loading fails loudly when the library has
not been built (python -m paper_2607_07432_amd.build).
"""
import ctypes
import os

import numpy as np

from . import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'liblbmib.so')

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_HIP, LBM_E_STATE, LBM_E_NONFINITE = 0, -1, -2, -3, -4, -5
F32, F64 = 32, 64
SWEEP_FUSED, SWEEP_THREE_PASS = 0, 1
BC_PERIODIC, BC_INFLOW_OUTFLOW, BC_CHARACTERISTIC = 0, 1, 2

EXPORTS = ['lbm_workspace_bytes', 'lbm_init_grid', 'ib_set_markers', 'lbm_step', 'lbm_step_timed',
           'ib_wall_loads', 'ib_wall_loads_noalloc', 'lbm_fields',
           'lbm_set_fields', 'lbm_get_state', 'lbm_set_state', 'lbm_residual', 'ib_geometry_counts',
           'ib_geometry', 'ib_marker_state', 'lbm_destroy', 'lbm_last_error', 'lbm_stream_copy',
           'lbm_batch_workspace_bytes', 'lbm_batch_create', 'lbm_batch_step', 'lbm_batch_step_timed',
           'lbm_batch_set_tile', 'lbm_batch_config', 'lbm_batch_residuals', 'lbm_batch_destroy', 'lbm_batch_last_error',
           'lbm_refine_create', 'lbm_refine_prolong', 'lbm_refine_step', 'lbm_refine_nest', 'lbm_refine_destroy',
           'lbm_refine_last_error',
           'lbm_learn_input', 'lbm_learn_target', 'lbm_learn_warm_start',
           'nn_unet_param_count', 'nn_unet_workspace_bytes', 'nn_unet_create', 'nn_unet_set_params',
           'nn_unet_get_params', 'nn_unet_get_grads', 'nn_unet_forward', 'nn_unet_backward', 'nn_unet_adam', 'nn_unet_clip_grad_norm',
           'nn_unet_destroy', 'nn_unet_last_error']


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'{msg} (code {code})')
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [('dim', ctypes.c_int), ('nx', ctypes.c_int), ('ny', ctypes.c_int), ('nz', ctypes.c_int),
                ('precision', ctypes.c_int), ('bc_x', ctypes.c_int), ('kernel', ctypes.c_int),
                ('max_markers', ctypes.c_int), ('with_aC', ctypes.c_int), ('sweep', ctypes.c_int),
                ('gamma', ctypes.c_double), ('mu', ctypes.c_double), ('lambda_', ctypes.c_double),
                ('sigma', ctypes.c_double), ('rho_inf', ctypes.c_double), ('u_inf', ctypes.c_double * 3),
                ('T_inf', ctypes.c_double), ('ref_len', ctypes.c_double), ('ref_area', ctypes.c_double),
                ('surface', ctypes.c_double), ('T_wall', ctypes.c_double), ('sigma_c', ctypes.c_double)]


class Loads(ctypes.Structure):
    _fields_ = [('F', ctypes.c_double * 3), ('Q_heat', ctypes.c_double), ('Cd', ctypes.c_double),
                ('Cl', ctypes.c_double), ('Nu', ctypes.c_double), ('eps_dir', ctypes.c_double),
                ('eps_neu', ctypes.c_double), ('eps_iso', ctypes.c_double), ('n_inactive', ctypes.c_int),
                ('n_markers', ctypes.c_int)]


_lib = None


def load_library(path=LIB_PATH):
    """Load liblbmib.so and declare its signatures. Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f'HIP library not built: {path} is missing '
                           '(run python -m paper_2607_07432_amd.build)')
    lib = ctypes.CDLL(path)
    P, vp, i, d = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    dp, ip, llp = P(d), P(i), P(ctypes.c_longlong)
    lib.lbm_workspace_bytes.argtypes = [P(Params)]
    lib.lbm_workspace_bytes.restype = ctypes.c_size_t
    lib.lbm_init_grid.argtypes = [P(Params), vp, ctypes.c_size_t, vp, P(vp)]
    lib.ib_set_markers.argtypes = [vp, i, dp, dp, dp, dp, ip, dp, i]
    lib.lbm_step.argtypes = [vp, i]
    lib.lbm_step_timed.argtypes = [vp, i, dp]
    lib.ib_wall_loads.argtypes = [vp, P(Loads)]
    lib.ib_wall_loads_noalloc.argtypes = [vp, P(Loads)]
    lib.lbm_fields.argtypes = [vp, i, i, vp, vp, vp, vp]
    lib.lbm_set_fields.argtypes = [vp, i, dp, dp, dp]
    lib.lbm_get_state.argtypes = [vp, dp, dp, dp]
    lib.lbm_set_state.argtypes = [vp, dp, dp, dp]
    lib.lbm_residual.argtypes = [vp, dp]
    lib.ib_geometry_counts.argtypes = [vp, llp]
    lib.ib_geometry.argtypes = [vp, llp, llp, dp, dp, dp, dp, dp, llp, llp, llp, dp, llp]
    lib.ib_marker_state.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_batch_workspace_bytes.argtypes = [P(vp), i]
    lib.lbm_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.lbm_batch_create.argtypes = [P(vp), i, vp, ctypes.c_size_t, i, P(vp)]
    lib.lbm_batch_step.argtypes = [vp, i]
    lib.lbm_batch_step_timed.argtypes = [vp, i, dp]
    lib.lbm_batch_config.argtypes = [vp, ip]
    lib.lbm_batch_set_tile.argtypes = [vp, i, i]
    lib.lbm_batch_residuals.argtypes = [vp, dp]
    lib.lbm_batch_destroy.argtypes = [vp]
    lib.lbm_batch_destroy.restype = None
    lib.lbm_batch_last_error.argtypes = [vp]
    lib.lbm_batch_last_error.restype = ctypes.c_char_p
    lib.lbm_refine_create.argtypes = [vp, vp, ip, i, i, P(vp)]
    lib.lbm_refine_prolong.argtypes = [vp]
    lib.lbm_refine_step.argtypes = [vp, i]
    lib.lbm_refine_nest.argtypes = [vp, vp]
    lib.lbm_refine_destroy.argtypes = [vp]
    lib.lbm_refine_destroy.restype = None
    lib.lbm_refine_last_error.argtypes = [vp]
    lib.lbm_refine_last_error.restype = ctypes.c_char_p
    fp = P(ctypes.c_float)
    lib.lbm_learn_input.argtypes = [vp, d, d, d, vp]
    lib.lbm_learn_target.argtypes = [vp, vp]
    lib.lbm_learn_warm_start.argtypes = [vp, vp]
    lib.nn_unet_param_count.argtypes = []
    lib.nn_unet_param_count.restype = ctypes.c_longlong
    lib.nn_unet_workspace_bytes.argtypes = [i, i, i]
    lib.nn_unet_workspace_bytes.restype = ctypes.c_size_t
    lib.nn_unet_create.argtypes = [i, i, i, vp, ctypes.c_size_t, vp, P(vp)]
    lib.nn_unet_set_params.argtypes = [vp, vp, i]
    lib.nn_unet_get_params.argtypes = [vp, vp, i]
    lib.nn_unet_get_grads.argtypes = [vp, vp, i]
    lib.nn_unet_forward.argtypes = [vp, i, vp, vp]
    lib.nn_unet_backward.argtypes = [vp, vp, vp, vp]
    lib.nn_unet_adam.argtypes = [vp, d, d, d, d, i, d]
    lib.nn_unet_clip_grad_norm.argtypes = [vp, d, vp]
    lib.nn_unet_destroy.argtypes = [vp]
    lib.nn_unet_destroy.restype = None
    lib.nn_unet_last_error.argtypes = [vp]
    lib.nn_unet_last_error.restype = ctypes.c_char_p
    for name in ('lbm_learn_input', 'lbm_learn_target', 'lbm_learn_warm_start', 'nn_unet_create',
                 'nn_unet_set_params', 'nn_unet_get_params', 'nn_unet_get_grads', 'nn_unet_forward',
                 'nn_unet_backward', 'nn_unet_adam', 'nn_unet_clip_grad_norm'):
        getattr(lib, name).restype = i
    del fp
    for name in ('lbm_init_grid', 'ib_set_markers', 'lbm_step', 'lbm_step_timed', 'ib_wall_loads', 'lbm_fields', 'lbm_set_fields',
                 'lbm_get_state', 'lbm_set_state', 'lbm_residual', 'ib_geometry_counts', 'ib_geometry',
                 'ib_marker_state', 'lbm_batch_create', 'lbm_batch_step', 'lbm_batch_step_timed',
                 'lbm_batch_config', 'lbm_batch_set_tile', 'lbm_batch_residuals'):
        getattr(lib, name).restype = i
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def _llptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)) if a is not None else None


def params_from_case(case, precision=F64, max_markers=None, with_aC=True, sweep=0):
    p = Params()
    p.dim = case.dim
    p.nx, p.ny = case.dims[0], case.dims[1]
    p.nz = case.dims[2] if case.dim == 3 else 1
    p.precision = precision
    p.bc_x = {'inflow_outflow': BC_INFLOW_OUTFLOW, 'characteristic': BC_CHARACTERISTIC}.get(case.bc, BC_PERIODIC)
    p.sigma_c = getattr(case, 'sigma_c', 0.25)
    p.kernel = case.kernel
    m = len(case.X) if case.X is not None else 0
    p.max_markers = max_markers if max_markers is not None else max(m, 1)
    p.with_aC = 1 if with_aC else 0
    p.sweep = sweep
    p.gamma, p.mu, p.lambda_, p.sigma = case.gamma, case.mu, case.lam, case.sigma
    p.rho_inf = case.rho_inf
    for a in range(3):
        p.u_inf[a] = case.u_inf[a] if a < len(case.u_inf) else 0.0
    p.T_inf = case.T_inf
    p.ref_len, p.ref_area, p.surface, p.T_wall = case.ref_len, case.ref_area, case.surface, case.T_wall
    return p


class Solver:
    """One grid on one GPU: a handle of the HIP library plus its torch-allocated workspace."""

    def __init__(self, params, device='cuda:0', stream=None):
        import torch
        self.lib = load_library()
        self.p = params
        self.D = params.dim
        self.Q = 9 if self.D == 2 else 19
        self.dims = (params.nx, params.ny, params.nz)
        self.N = params.nx * params.ny * params.nz
        self.device = torch.device(device)
        nbytes = self.lib.lbm_workspace_bytes(ctypes.byref(params))
        if nbytes == 0:
            raise LbmError(LBM_E_INVAL, 'invalid parameters')
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self.lib.lbm_init_grid(ctypes.byref(params), ctypes.c_void_p(self._ws_ptr), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_last_error(None).decode())
        self.h = h
        self.m = 0

    @classmethod
    def from_case(cls, case, precision=F64, max_markers=None, with_aC=True, device='cuda:0', markers=True,
                  sweep=0):
        s = cls(params_from_case(case, precision, max_markers, with_aC, sweep), device)
        if markers and case.X is not None:
            s.set_markers(case.X, case.n, case.u_wall, case.t_kind, case.t_value, case.method)
        return s

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, 'h', None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_markers(self, X, n, u_wall, t_kind, t_value, method=workloads.METHOD_FODIBM_R, area_w=None):
        X = np.ascontiguousarray(X, dtype=np.float64)
        n = np.ascontiguousarray(n, dtype=np.float64)
        u_wall = np.ascontiguousarray(u_wall, dtype=np.float64)
        t_kind = np.ascontiguousarray(t_kind, dtype=np.int32)
        t_value = np.ascontiguousarray(t_value, dtype=np.float64)
        aw = np.ascontiguousarray(area_w, dtype=np.float64) if area_w is not None else None
        m = len(X)
        self._check(self.lib.ib_set_markers(self.h, m, _dptr(X), _dptr(n), _dptr(aw), _dptr(u_wall),
                                            _iptr(t_kind), _dptr(t_value), int(method)))
        self.m = m

    def step(self, n=1):
        self._check(self.lib.lbm_step(self.h, int(n)))

    def step_timed(self, n):
        """n steps; returns the average per-step ms of (markers, spread, sweep) from HIP events."""
        ms = np.zeros(3)
        self._check(self.lib.lbm_step_timed(self.h, int(n), _dptr(ms)))
        return ms

    def residual(self):
        r = ctypes.c_double()
        self._check(self.lib.lbm_residual(self.h, ctypes.byref(r)))
        return r.value

    def loads(self, noalloc=False):
        """ib_wall_loads (noalloc=True: ib_wall_loads_noalloc, scratch in the library's static array)."""
        out = Loads()
        fn = self.lib.ib_wall_loads_noalloc if noalloc else self.lib.ib_wall_loads
        self._check(fn(self.h, ctypes.byref(out)))
        return dict(F=np.array(out.F[:self.D]), Q_heat=out.Q_heat, Cd=out.Cd, Cl=out.Cl, Nu=out.Nu,
                    eps_dir=out.eps_dir, eps_neu=out.eps_neu, eps_iso=out.eps_iso, n_inactive=out.n_inactive,
                    n_markers=out.n_markers)

    def fields(self, dtype=F64):
        """Host numpy fields (rho, u[D], T, p) on the grid shape (nz, ny, nx) / (ny, nx)."""
        npd = np.float64 if dtype == F64 else np.float32
        rho = np.empty(self.N, npd)
        u = np.empty(self.D * self.N, npd)
        T = np.empty(self.N, npd)
        p = np.empty(self.N, npd)
        vp = lambda a: ctypes.c_void_p(a.ctypes.data)
        self._check(self.lib.lbm_fields(self.h, dtype, 0, vp(rho), vp(u), vp(T), vp(p)))
        shape = self.grid_shape
        return rho.reshape(shape), u.reshape((self.D,) + shape), T.reshape(shape), p.reshape(shape)

    def fields_device(self, rho, u, T, p, dtype=F64):
        """Write fields into caller-owned torch tensors (stream ordered)."""
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        self._check(self.lib.lbm_fields(self.h, dtype, 1, ptr(rho), ptr(u), ptr(T), ptr(p)))

    @property
    def grid_shape(self):
        return (self.dims[1], self.dims[0]) if self.D == 2 else (self.dims[2], self.dims[1], self.dims[0])

    def set_fields(self, rho, u, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        self._check(self.lib.lbm_set_fields(self.h, 0, _dptr(rho), _dptr(u), _dptr(T)))

    def get_state(self):
        """Canonical FP64 state: f (Q, *grid), rhoE (*grid), H2 (D, D, *grid)."""
        f = np.empty(self.Q * self.N)
        e = np.empty(self.N)
        H2 = np.empty(self.D * self.D * self.N)
        self._check(self.lib.lbm_get_state(self.h, _dptr(f), _dptr(e), _dptr(H2)))
        shape = self.grid_shape
        return f.reshape((self.Q,) + shape), e.reshape(shape), H2.reshape((self.D, self.D) + shape)

    def set_state(self, f, rhoE, H2):
        f = np.ascontiguousarray(f, dtype=np.float64).ravel()
        e = np.ascontiguousarray(rhoE, dtype=np.float64).ravel()
        H2 = np.ascontiguousarray(H2, dtype=np.float64).ravel()
        self._check(self.lib.lbm_set_state(self.h, _dptr(f), _dptr(e), _dptr(H2)))

    def learn_input(self, out, sdf_scale, ma_n, re_n):
        """Network input planes [ny, nx, 4] (FP32 device tensor) of this case."""
        self._check(self.lib.lbm_learn_input(self.h, float(sdf_scale), float(ma_n), float(re_n),
                                             ctypes.c_void_p(out.data_ptr())))

    def learn_target(self, out):
        """Normalised fields [ny, nx, 4] (FP32 device tensor) of the current state."""
        self._check(self.lib.lbm_learn_target(self.h, ctypes.c_void_p(out.data_ptr())))

    def warm_start(self, pred):
        """Set the state to the equilibrium of a normalised prediction [ny, nx, 4] (FP32 device)."""
        self._check(self.lib.lbm_learn_warm_start(self.h, ctypes.c_void_p(pred.data_ptr())))

    def geometry(self):
        c = np.zeros(6, dtype=np.int64)
        self._check(self.lib.ib_geometry_counts(self.h, _llptr(c)))
        m, nrows, nent, nsupp, nint, nact = (int(v) for v in c)
        D = self.D
        out = dict(supp_ptr=np.zeros(m + 1, np.int64), supp_node=np.zeros(nsupp, np.int64),
                   supp_w=np.zeros(nsupp), phi=np.zeros(m), xstar=np.zeros(m * D), dbv=np.zeros(m),
                   W=np.zeros(m), rows=np.zeros(nrows, np.int64), row_ptr=np.zeros(nrows + 1, np.int64),
                   col_marker=np.zeros(nent, np.int64), col_s=np.zeros(nent), interior=np.zeros(nint, np.int64))
        self._check(self.lib.ib_geometry(self.h, _llptr(out['supp_ptr']), _llptr(out['supp_node']),
                                         _dptr(out['supp_w']), _dptr(out['phi']), _dptr(out['xstar']),
                                         _dptr(out['dbv']), _dptr(out['W']), _llptr(out['rows']),
                                         _llptr(out['row_ptr']), _llptr(out['col_marker']), _dptr(out['col_s']),
                                         _llptr(out['interior'])))
        out['xstar'] = out['xstar'].reshape(m, D)
        out['n_active'] = nact
        return out

    def marker_state(self):
        m, D = self.m, self.D
        F, Wib, Qib, rho, T, uP, TP = (np.zeros(m * D), np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m),
                                       np.zeros(m * D), np.zeros(m))
        self._check(self.lib.ib_marker_state(self.h, _dptr(F), _dptr(Wib), _dptr(Qib), _dptr(rho), _dptr(T),
                                             _dptr(uP), _dptr(TP)))
        return dict(F=F.reshape(m, D), Wib=Wib, Qib=Qib, rho=rho, T=T, uP=uP.reshape(m, D), TP=TP)


class Batch:
    """Independent 2D grids (Solver objects on one stream) advanced together by the batch API."""

    def __init__(self, solvers, autotune=True):
        import torch
        if not solvers:
            raise ValueError('empty batch')
        self.lib = load_library()
        self.solvers = list(solvers)
        n = len(self.solvers)
        arr = (ctypes.c_void_p * n)(*[s.h.value for s in self.solvers])
        self._arr = arr
        nbytes = self.lib.lbm_batch_workspace_bytes(arr, n)
        if nbytes == 0:
            raise LbmError(LBM_E_INVAL, 'invalid batch (2D cases of one precision on one stream)')
        dev = self.solvers[0].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = (self.workspace.data_ptr() + 255) & ~255
        b = ctypes.c_void_p()
        rc = self.lib.lbm_batch_create(arr, n, ctypes.c_void_p(ptr), nbytes, 1 if autotune else 0, ctypes.byref(b))
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_batch_last_error(None).decode())
        self.b = b
        self.nodes = sum(s.N for s in self.solvers)

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_batch_last_error(self.b).decode())
        return rc

    def step(self, n=1):
        self._check(self.lib.lbm_batch_step(self.b, int(n)))

    def step_timed(self, n):
        """n steps without graphs; returns the average per-step ms of (markers, spread, sweep)."""
        ms = np.zeros(3)
        self._check(self.lib.lbm_batch_step_timed(self.b, int(n), _dptr(ms)))
        return ms

    def set_tile(self, tile_x, chunk):
        self._check(self.lib.lbm_batch_set_tile(self.b, int(tile_x), int(chunk)))

    def config(self):
        c = np.zeros(6, dtype=np.int32)
        self._check(self.lib.lbm_batch_config(self.b, _iptr(c)))
        return dict(tile_x=int(c[0]), chunk=int(c[1]), grid=int(c[2]), items=int(c[3]), markers=int(c[4]),
                    rows=int(c[5]))

    def residuals(self):
        """Residual of every case after the last batch step (nan for a case whose state holds a
        non-finite value)."""
        out = np.empty(len(self.solvers))
        self._check(self.lib.lbm_batch_residuals(self.b, _dptr(out)))
        return out.tolist()

    def close(self):
        if getattr(self, 'b', None):
            self.lib.lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Refinement:
    """A fine Solver embedded in a coarse Solver (ratio 2; lbm_refine_* of the C ABI); couplings
    nest through `nest`.

    origin: coarse node of fine node 0 per axis (x, y[, z]). The fine solver must have been created
    with twice the coarse mu and lambda_ and periodic closure (fine_params_for builds them)."""

    def __init__(self, coarse, fine, origin, band=2, margin=8):
        self.lib = load_library()
        self.coarse, self.fine = coarse, fine
        org = np.ascontiguousarray(list(origin) + [0] * (3 - len(origin)), dtype=np.int32)
        r = ctypes.c_void_p()
        rc = self.lib.lbm_refine_create(coarse.h, fine.h, _iptr(org), int(band), int(margin), ctypes.byref(r))
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_refine_last_error(None).decode())
        self.r = r

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_refine_last_error(self.r).decode())
        return rc

    def prolong(self):
        """Every fine node from the current coarse state."""
        self._check(self.lib.lbm_refine_prolong(self.r))

    def step(self, n=1):
        self._check(self.lib.lbm_refine_step(self.r, int(n)))

    def nest(self, inner):
        """Advance this coupling's fine level through `inner` (a Refinement whose coarse solver is
        this one's fine solver); step the outermost coupling only."""
        self._check(self.lib.lbm_refine_nest(self.r, inner.r))
        self.inner = inner

    def residual(self):
        """Coarse residual of the last coupled step (restriction included)."""
        return self.coarse.residual()

    def close(self):
        if getattr(self, 'r', None):
            self.lib.lbm_refine_destroy(self.r)
            self.r = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fine_params_for(coarse_params, fine_cells, max_markers=1):
    """Parameters of the fine level of a block of fine_cells[a] coarse cells per axis: 2 fine_cells[a]
    nodes, twice the coarse mu and lambda_, periodic closure, the coarse gas and free stream."""
    p = Params()
    ctypes.memmove(ctypes.byref(p), ctypes.byref(coarse_params), ctypes.sizeof(Params))
    p.nx = 2 * fine_cells[0]
    p.ny = 2 * fine_cells[1]
    p.nz = 2 * fine_cells[2] if coarse_params.dim == 3 else 1
    p.mu = 2.0 * coarse_params.mu
    p.lambda_ = 2.0 * coarse_params.lambda_
    p.bc_x = BC_PERIODIC
    p.max_markers = max_markers
    return p


NN_OK = 0


class UNet:
    """The neural operator of the learned warm start (batch capacity, H x W images) on one GPU."""

    def __init__(self, batch, H, W, device='cuda:0', stream=None):
        import torch
        self.lib = load_library()
        self.B, self.H, self.W = batch, H, W
        self.device = torch.device(device)
        self.n_params = int(self.lib.nn_unet_param_count())
        nbytes = self.lib.nn_unet_workspace_bytes(batch, H, W)
        if nbytes == 0:
            raise LbmError(LBM_E_INVAL, 'invalid network size (H % 16, W % 128)')
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        u = ctypes.c_void_p()
        rc = self.lib.nn_unet_create(batch, H, W, ctypes.c_void_p(ptr), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(u))
        if rc != NN_OK:
            raise LbmError(rc, self.lib.nn_unet_last_error(None).decode())
        self.u = u
        self.loss_buf = torch.zeros(2, dtype=torch.float64, device=self.device)
        self.norm_buf = torch.zeros(2, dtype=torch.float64, device=self.device)

    def _check(self, rc):
        if rc != NN_OK:
            raise LbmError(rc, self.lib.nn_unet_last_error(self.u).decode())

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == self.n_params
        self._check(self.lib.nn_unet_set_params(self.u, ctypes.c_void_p(theta.ctypes.data), 0))

    def get_params(self):
        out = np.empty(self.n_params, np.float32)
        self._check(self.lib.nn_unet_get_params(self.u, ctypes.c_void_p(out.ctypes.data), 0))
        return out

    def get_grads(self):
        out = np.empty(self.n_params, np.float32)
        self._check(self.lib.nn_unet_get_grads(self.u, ctypes.c_void_p(out.ctypes.data), 0))
        return out

    def forward(self, x, out=None):
        """x: FP32 device tensor [b, H, W, 4]; returns (or fills) the FP32 output [b, H, W, 4]."""
        import torch
        b = x.shape[0]
        if out is None:
            out = torch.empty((b, self.H, self.W, 4), dtype=torch.float32, device=self.device)
        self._check(self.lib.nn_unet_forward(self.u, b, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr())))
        return out

    def backward(self, target, mask=None):
        """Gradient of the masked MSE of the last forward; returns the device loss buffer {L, count}."""
        mp = ctypes.c_void_p(mask.data_ptr()) if mask is not None else None
        self._check(self.lib.nn_unet_backward(self.u, ctypes.c_void_p(target.data_ptr()), mp,
                                              ctypes.c_void_p(self.loss_buf.data_ptr())))
        return self.loss_buf

    def clip_grad_norm(self, max_norm):
        """Scale the gradient to global L2 norm <= max_norm; returns the device buffer
        {norm before clipping, applied scale}."""
        self._check(self.lib.nn_unet_clip_grad_norm(self.u, float(max_norm), ctypes.c_void_p(self.norm_buf.data_ptr())))
        return self.norm_buf

    def adam(self, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        self._check(self.lib.nn_unet_adam(self.u, float(lr), float(beta1), float(beta2), float(eps), int(t),
                                          float(weight_decay)))

    def close(self):
        if getattr(self, 'u', None):
            self.lib.nn_unet_destroy(self.u)
            self.u = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
