"""Thin ctypes binding of libstfd.so (include/stfd.h): argument marshalling only.

Device vectors are torch.complex128 CUDA tensors (interleaved re/im doubles,
time index fastest, right-hand sides stacked slowest); streams are torch
streams.  Every computation happens in the library's HIP kernels; if the
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstfd.so")

OK, NOT_CONVERGED, EINVAL, ENOTSPD, EBREAKDOWN, ENOMEM, EHIP = 0, 1, -1, -2, -3, -4, -5
FP64, FP32, BF16 = 0, 1, 2
GEOM_UNIT_CUBE, GEOM_QUARTER_ANNULUS = 0, 1
PRECOND_AUTO, PRECOND_PARAMETRIC = 0, 1
MATVEC_AUTO, MATVEC_STENCIL, MATVEC_SUMFAC = 0, 1, 2
TIME_INITIAL, TIME_FINAL = 0, 1  # least-squares method / ultraweak method (Section 4.4)
SHIFT_NONE, SHIFT_MEAN_POTENTIAL = 0, 1  # preconditioner without / with the mean potential
X0_ZERO, X0_GIVEN, PCG_GRAPH, X0_SCALED = 0, 1, 2, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}


class SetupDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("p_t", ctypes.c_int), ("p_s", ctypes.c_int),
                ("knots_t", ctypes.POINTER(ctypes.c_double)), ("n_knots_t", ctypes.c_int),
                ("knots_s", ctypes.POINTER(ctypes.c_double) * 3), ("n_knots_s", ctypes.c_int * 3),
                ("T", ctypes.c_double), ("nu", ctypes.c_double),
                ("V_quad", ctypes.POINTER(ctypes.c_double)), ("n_quad", ctypes.c_int),
                ("max_nrhs", ctypes.c_int), ("geometry", ctypes.c_int), ("geom", ctypes.c_double * 2),
                ("precond", ctypes.c_int), ("matvec", ctypes.c_int), ("no_rhs_workspace", ctypes.c_int),
                ("time_condition", ctypes.c_int), ("autotune", ctypes.c_int), ("precond_shift", ctypes.c_int),
                ("fused_segment_length", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("autotuned", ctypes.c_int), ("mode_product_row_groups", (ctypes.c_int * 3) * 3),
                ("time_segment_length", ctypes.c_int), ("time_transfers_in_kernel", ctypes.c_int),
                ("tune_ms", ctypes.c_double), ("time_factors_in_kernel", ctypes.c_int),
                ("fused_time", ctypes.c_int), ("fused_segment_length", ctypes.c_int),
                ("fused_factors_in_kernel", ctypes.c_int)]


class PcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double), ("x0_scale", ctypes.c_double)]


class FnoDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("c_in", ctypes.c_int), ("width", ctypes.c_int),
                ("modes1", ctypes.c_int), ("modes2", ctypes.c_int), ("layers", ctypes.c_int), ("proj", ctypes.c_int),
                ("c_out", ctypes.c_int), ("max_batch", ctypes.c_int), ("seed", ctypes.c_uint64)]


class StfdError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib().stfd_strerror(code).decode()
        if code == EHIP:
            msg += f" (hip error {_lib().stfd_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")


_LIB = None

# exported symbols and their signatures (mirrors include/stfd.h)
_VP, _DP, _IP, _I64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_int64
_FP = ctypes.POINTER(ctypes.c_float)
SIGNATURES = {
    "stfd_quad_points": (ctypes.c_int, [_DP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _DP, _DP, _IP]),
    "stfd_setup": (ctypes.c_int, [ctypes.POINTER(SetupDesc), ctypes.POINTER(_VP)]),
    "stfd_sizes": (ctypes.c_int, [_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "stfd_apply_preconditioner": (ctypes.c_int, [_VP, _VP, _VP, _I64, ctypes.c_int, _VP]),
    "stfd_matvec": (ctypes.c_int, [_VP, _VP, _VP, _I64, _VP]),
    "stfd_apply_preconditioner_static": (ctypes.c_int, [_VP, _VP, _VP, _I64, ctypes.c_int, _VP]),
    "stfd_pcg_solve": (ctypes.c_int, [_VP, _VP, _VP, _I64, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(PcgInfo), _VP]),
    "stfd_get_pencil": (ctypes.c_int, [_VP, ctypes.c_int, _DP, _DP]),
    "stfd_get_tuning": (ctypes.c_int, [_VP, _VP]),
    "stfd_set_tuning": (ctypes.c_int, [_VP, _VP]),
    "stfd_get_precond_shift": (ctypes.c_int, [_VP, _DP]),
    "stfd_load_vector": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(_VP), _VP, _DP, _I64, _VP]),
    "stfd_update_potential": (ctypes.c_int, [_VP, _DP, _VP]),
    "stfd_set_lift_max_iterations": (ctypes.c_int, [_VP, ctypes.c_int]),
    "stfd_timing_begin": (ctypes.c_int, [_VP, ctypes.c_int]),
    "stfd_timing_end": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "stfd_time_mode_product": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP,
                                              ctypes.POINTER(ctypes.c_double)]),
    "stfd_fno_create": (ctypes.c_int, [ctypes.POINTER(FnoDesc), ctypes.POINTER(_VP)]),
    "stfd_fno_num_params": (ctypes.c_int, [_VP, ctypes.POINTER(_I64)]),
    "stfd_fno_get_params": (ctypes.c_int, [_VP, _FP]),
    "stfd_fno_set_params": (ctypes.c_int, [_VP, _FP]),
    "stfd_fno_get_grads": (ctypes.c_int, [_VP, _FP]),
    "stfd_fno_forward": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP]),
    "stfd_fno_backward": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP]),
    "stfd_fno_rel_l2": (ctypes.c_int, [_VP, _VP, _I64, ctypes.c_int, _VP, _FP, _VP]),
    "stfd_fno_adam_step": (ctypes.c_int, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP]),
    "stfd_fno_to_f64": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "stfd_fno_diff_f64": (ctypes.c_int, [_VP, _VP, _VP, _I64, _VP]),
    "stfd_fno_energy_loss": (ctypes.c_int, [_VP, _VP, _VP, _I64, ctypes.c_int, _VP, _DP, _FP, _VP]),
    "stfd_fno_destroy": (None, [_VP]),
    "stfd_map_points": (ctypes.c_int, [_VP, _DP, _I64, _DP]),
    "stfd_pcg_solve_batched": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(_VP),
                                              ctypes.POINTER(_VP), ctypes.POINTER(_I64), ctypes.c_double,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(PcgInfo),
                                              _VP]),
    "stfd_destroy": (None, [_VP]),
    "stfd_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "stfd_last_hip_error": (ctypes.c_int, []),
    "stfd_debug_mfma_layout": (ctypes.c_int, [_DP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
}


def _lib():
    global _LIB
    if _LIB is None:
        # Load torch first so that the library binds to the HIP runtime torch already
        # loaded; two runtimes in one process do not see the same devices.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_18461_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(code, where, allow=(OK,)):
    if code not in allow:
        raise StfdError(code, where)
    return code


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def quad_points(knots, degree: int, n_quad: int = 0, scale: float = 1.0):
    """Element-wise Gauss points/weights of the library on an open knot vector (scaled)."""
    kn = np.ascontiguousarray(knots, dtype=np.float64)
    n = ctypes.c_int(0)
    _check(_lib().stfd_quad_points(_dptr(kn), len(kn), degree, n_quad, scale, None, None, ctypes.byref(n)),
           "stfd_quad_points")
    pts, wts = np.empty(n.value), np.empty(n.value)
    _check(_lib().stfd_quad_points(_dptr(kn), len(kn), degree, n_quad, scale, _dptr(pts), _dptr(wts),
                                   ctypes.byref(n)), "stfd_quad_points")
    return pts, wts


def sample_on_quad_grid(fn, knots_s, p_s: int, n_quad: int = 0) -> np.ndarray:
    """fn(x_1, ..., x_d) on the library's spatial tensor Gauss grid, flattened x_1 fastest."""
    pts = [quad_points(k, p_s, n_quad)[0] for k in knots_s]
    grids = np.meshgrid(*reversed(pts), indexing="ij")
    vals = np.asarray(fn(*reversed(grids)), dtype=np.float64)
    return np.ascontiguousarray(vals.ravel())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, n_expected, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor")
    if t.numel() != n_expected:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n_expected}")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """Handle of one set-up problem (stfd_setup / stfd_destroy)."""

    def __init__(self, knots_t, knots_s, p_t: int, p_s: int, T: float = 1.0, nu: float = 1.0,
                 V_quad=None, n_quad: int = 0, max_nrhs: int = 1, geometry=GEOM_UNIT_CUBE, radii=(1.0, 2.0),
                 precond=PRECOND_AUTO, rhs_workspace: bool = True, matvec=MATVEC_AUTO,
                 time_condition=TIME_INITIAL, autotune: bool = False, precond_shift=SHIFT_NONE,
                 fused_segment_length: int = 0):
        d = len(knots_s)
        self._keep = [np.ascontiguousarray(knots_t, dtype=np.float64)]
        desc = SetupDesc()
        desc.d, desc.p_t, desc.p_s = d, p_t, p_s
        desc.knots_t, desc.n_knots_t = _dptr(self._keep[0]), len(self._keep[0])
        for l in range(3):
            if l < d:
                k = np.ascontiguousarray(knots_s[l], dtype=np.float64)
                self._keep.append(k)
                desc.knots_s[l], desc.n_knots_s[l] = _dptr(k), len(k)
            else:
                desc.knots_s[l], desc.n_knots_s[l] = None, 0
        desc.T, desc.nu = T, nu
        if V_quad is not None:
            v = np.ascontiguousarray(V_quad, dtype=np.float64)
            self._keep.append(v)
            desc.V_quad = _dptr(v)
        else:
            desc.V_quad = None
        desc.n_quad, desc.max_nrhs = n_quad, max_nrhs
        desc.geometry = geometry
        desc.geom[0], desc.geom[1] = radii
        desc.precond = precond
        desc.no_rhs_workspace = 0 if rhs_workspace else 1
        desc.time_condition = time_condition
        desc.autotune = 1 if autotune else 0
        desc.precond_shift = precond_shift
        desc.fused_segment_length = fused_segment_length
        desc.matvec = matvec
        h = ctypes.c_void_p()
        self._h = None
        _check(_lib().stfd_setup(ctypes.byref(desc), ctypes.byref(h)), "stfd_setup")
        self._h = h
        nt, ns, nd = ctypes.c_int64(), (ctypes.c_int64 * 3)(), ctypes.c_int64()
        _check(_lib().stfd_sizes(self._h, ctypes.byref(nt), ns, ctypes.byref(nd)), "stfd_sizes")
        self.d, self.n_t, self.n_s, self.N = d, nt.value, [ns[i] for i in range(d)], nd.value
        self.N_s = self.N // self.n_t
        self.max_nrhs = max_nrhs
        # Gauss grids of the load vector: time (scaled by T), then x_1 .. x_d
        self.quad = [quad_points(knots_t, p_t, n_quad, T)] + [quad_points(k, p_s, n_quad) for k in knots_s]
        self.m_full = [self.n_t + 1] + [n + 2 for n in self.n_s]

    def close(self):
        if self._h is not None and _LIB is not None:
            _LIB.stfd_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def precond_shift(self):
        """stfd_get_precond_shift: the constant c of the preconditioner (0 without a shift)."""
        c = ctypes.c_double()
        _check(_lib().stfd_get_precond_shift(self._h, ctypes.byref(c)), "stfd_get_precond_shift")
        return c.value

    def get_tuning(self):
        """stfd_get_tuning: the launch shapes in use (timed at setup when autotune was set)."""
        t = Tuning()
        _check(_lib().stfd_get_tuning(self._h, ctypes.byref(t)), "stfd_get_tuning")
        return {"autotuned": bool(t.autotuned),
                "mode_product_row_groups": {name: [t.mode_product_row_groups[k][l] for l in range(self.d)]
                                            for k, name in enumerate(("fp64", "fp32", "bf16"))},
                "time_segment_length": t.time_segment_length,
                "time_transfers_in_kernel": bool(t.time_transfers_in_kernel),
                "time_factors_in_kernel": bool(t.time_factors_in_kernel), "tune_ms": t.tune_ms,
                "fused_time": bool(t.fused_time), "fused_segment_length": t.fused_segment_length,
                "fused_factors_in_kernel": bool(t.fused_factors_in_kernel)}

    def set_mode_product_shapes(self, shapes):
        """stfd_set_tuning: {"fp64"|"fp32"|"bf16": [shape per direction]} (1, 2 = row groups per wave of
        the one-group form, 3 = the wide form); the time-solve fields are kept."""
        t = Tuning()
        _check(_lib().stfd_get_tuning(self._h, ctypes.byref(t)), "stfd_get_tuning")
        for k, name in enumerate(("fp64", "fp32", "bf16")):
            for l, v in enumerate(shapes.get(name, [t.mode_product_row_groups[k][l] for l in range(self.d)])):
                t.mode_product_row_groups[k][l] = int(v)
        return _check(_lib().stfd_set_tuning(self._h, ctypes.byref(t)), "stfd_set_tuning")

    def set_fused_time(self, on: bool):
        """stfd_set_tuning: run the last direction's products and the time solves as one launch (on)
        or as separate launches; the other fields are kept."""
        t = Tuning()
        _check(_lib().stfd_get_tuning(self._h, ctypes.byref(t)), "stfd_get_tuning")
        t.fused_time = 1 if on else 0
        return _check(_lib().stfd_set_tuning(self._h, ctypes.byref(t)), "stfd_set_tuning")

    def get_pencil(self, l: int):
        n = self.n_s[l]
        U, lam = np.empty((n, n)), np.empty(n)
        _check(_lib().stfd_get_pencil(self._h, l, _dptr(U), _dptr(lam)), "stfd_get_pencil")
        return U, lam

    def grid_shape(self, axes):
        """Sample counts of the Gauss grid over the listed axes (0 = time, l + 1 = x_l), fastest first."""
        return [len(self.quad[a][0]) for a in axes]

    def face_axes(self, l: int):
        """Axes of the face x_l = const, fastest first: time, then x_k for k != l."""
        return [0] + [k + 1 for k in range(self.d) if k != l]

    def map_points(self, xi):
        """Physical coordinates of parametric points xi (n x d)."""
        xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, self.d)
        x = np.empty_like(xi)
        _check(_lib().stfd_map_points(self._h, _dptr(xi), xi.shape[0], _dptr(x)), "stfd_map_points")
        return x

    def physical_grid(self):
        """Physical coordinates (x_1, ..., x_d) of the spatial Gauss grid, each flattened x_1 fastest."""
        g = self._grid(range(1, self.d + 1))
        xi = np.stack([a.ravel() for a in g], axis=1)
        x = self.map_points(xi)
        return [x[:, l] for l in range(self.d)]

    def update_potential(self, V_quad=None, stream=None):
        """stfd_update_potential: replace V (samples on the spatial Gauss grid, x_1 fastest)."""
        v = np.ascontiguousarray(V_quad, dtype=np.float64) if V_quad is not None else None
        _check(_lib().stfd_update_potential(self._h, _dptr(v) if v is not None else None, _stream_ptr(stream)),
               "stfd_update_potential")

    def _grid(self, axes):
        """Coordinate arrays of the Gauss grid over `axes` (fastest first), in C order (slowest first)."""
        pts = [self.quad[a][0] for a in axes]
        return list(reversed(np.meshgrid(*reversed(pts), indexing="ij")))

    def sample_spacetime(self, fn):
        """fn(t, x_1, ..., x_d) on the space-time grid, flattened time fastest (complex128)."""
        g = self._grid(range(self.d + 1))
        return np.array(np.broadcast_to(fn(*g), g[0].shape), dtype=np.complex128).ravel()

    def sample_space(self, fn):
        """fn(x_1, ..., x_d) on the spatial grid, flattened x_1 fastest (complex128)."""
        g = self._grid(range(1, self.d + 1))
        return np.array(np.broadcast_to(fn(*g), g[0].shape), dtype=np.complex128).ravel()

    def sample_faces(self, fn):
        """fn(t, x_1, ..., x_d) on the 2d lateral faces (x_l = 0, then x_l = 1, for each l)."""
        out = []
        for l in range(self.d):
            g = self._grid(self.face_axes(l))
            for side in (0.0, 1.0):
                coords, j = [g[0]], 1
                for k in range(self.d):
                    if k == l:
                        coords.append(np.full_like(g[0], side))
                    else:
                        coords.append(g[j])
                        j += 1
                out.append(np.array(np.broadcast_to(fn(*coords), g[0].shape), dtype=np.complex128).ravel())
        return out

    def load_vector(self, fbar, f_q=None, u0_q=None, dirichlet_q=None, nrhs: int = 1, stream=None,
                    return_lift: bool = False):
        """stfd_load_vector: fbar (device, N * nrhs complex128) <- right-hand side with lifting.

        f_q: space-time samples (time fastest), u0_q: spatial samples (x_1 fastest),
        dirichlet_q: None or 2 d face samples (x_l = 0, x_l = 1 for each l; entries may be None);
        all contiguous complex128 device tensors with nrhs samples stacked.
        Returns the lifting tensors (host, nrhs x prod m_full, time fastest) if return_lift.
        """
        n_grid = int(np.prod(self.grid_shape(range(self.d + 1))))
        n_sp = int(np.prod(self.grid_shape(range(1, self.d + 1))))
        fq = _dev_ptr(f_q, n_grid * nrhs, "f_q") if f_q is not None else None
        u0 = _dev_ptr(u0_q, n_sp * nrhs, "u0_q") if u0_q is not None else None
        faces = None
        if dirichlet_q is not None:
            if len(dirichlet_q) != 2 * self.d:
                raise ValueError("dirichlet_q needs 2 d face arrays")
            faces = (_VP * (2 * self.d))()
            for k, a in enumerate(dirichlet_q):
                if a is not None:
                    n_face = int(np.prod(self.grid_shape(self.face_axes(k // 2))))
                    faces[k] = _dev_ptr(a, n_face * nrhs, f"dirichlet_q[{k}]").value
        lift = np.zeros(int(np.prod(self.m_full)) * nrhs, dtype=np.complex128) if return_lift else None
        _check(_lib().stfd_load_vector(self._h, fq, u0, faces, _dev_ptr(fbar, self.N * nrhs, "fbar"),
                                       lift.ctypes.data_as(_DP) if lift is not None else None, nrhs,
                                       _stream_ptr(stream)), "stfd_load_vector")
        return lift

    def timing_begin(self, capacity: int = 1024):
        """stfd_timing_begin: HIP events around every mode-product launch of the applies that follow."""
        return _check(_lib().stfd_timing_begin(self._h, int(capacity)), "stfd_timing_begin")

    def timing_end(self):
        """stfd_timing_end: (summed event time in ms, launches recorded) of the mode products."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(_lib().stfd_timing_end(self._h, ctypes.byref(ms), ctypes.byref(n)), "stfd_timing_end")
        return ms.value, n.value

    def time_mode_product(self, direction: int = 0, precision=FP64, reps: int = 200, stream=None):
        """stfd_time_mode_product: average ms per launch of the forward mode product of one
        direction, launched reps times back to back."""
        precision = PRECISIONS.get(precision, precision)
        ms = ctypes.c_double()
        _check(_lib().stfd_time_mode_product(self._h, int(direction), precision, int(reps), _stream_ptr(stream),
                                             ctypes.byref(ms)), "stfd_time_mode_product")
        return ms.value

    def set_lift_max_iterations(self, max_iter: int):
        """stfd_set_lift_max_iterations: iteration limit of the lifting CG in load_vector."""
        return _check(_lib().stfd_set_lift_max_iterations(self._h, int(max_iter)), "stfd_set_lift_max_iterations")

    def apply_preconditioner(self, r, s, nrhs: int = 1, precision=FP64, stream=None):
        precision = PRECISIONS.get(precision, precision)
        return _check(_lib().stfd_apply_preconditioner(self._h, _dev_ptr(r, self.N * nrhs, "r"),
                                                       _dev_ptr(s, self.N * nrhs, "s"), nrhs, precision,
                                                       _stream_ptr(stream)), "stfd_apply_preconditioner")

    def apply_preconditioner_static(self, r, s, nrhs: int = 1, precision=FP64, stream=None):
        """stfd_apply_preconditioner_static: the apply with the library's fixed device scratch."""
        precision = PRECISIONS.get(precision, precision)
        return _check(_lib().stfd_apply_preconditioner_static(self._h, _dev_ptr(r, self.N * nrhs, "r"),
                                                              _dev_ptr(s, self.N * nrhs, "s"), nrhs, precision,
                                                              _stream_ptr(stream)),
                      "stfd_apply_preconditioner_static")

    def matvec(self, x, y, nrhs: int = 1, stream=None):
        return _check(_lib().stfd_matvec(self._h, _dev_ptr(x, self.N * nrhs, "x"), _dev_ptr(y, self.N * nrhs, "y"),
                                         nrhs, _stream_ptr(stream)), "stfd_matvec")

    def pcg_solve(self, f, u, nrhs: int = 1, rtol: float = 1e-8, maxit: int = 200, x0_given: bool = False,
                  precision=FP64, stream=None, check=True, graph: bool = False, x0_scaled: bool = False):
        precision = PRECISIONS.get(precision, precision)
        info = (PcgInfo * nrhs)()
        flags = (X0_GIVEN if x0_given else X0_ZERO) | (PCG_GRAPH if graph else 0)
        if x0_scaled:
            flags |= X0_GIVEN | X0_SCALED
        rc = _lib().stfd_pcg_solve(self._h, _dev_ptr(f, self.N * nrhs, "f"), _dev_ptr(u, self.N * nrhs, "u"),
                                   nrhs, rtol, maxit, flags, precision, info, _stream_ptr(stream))
        if check:
            _check(rc, "stfd_pcg_solve", allow=(OK, NOT_CONVERGED))
        return rc, _infos(info)


def _infos(info):
    return [dict(iters=i.iters, status=i.status, rel_res=i.rel_res, true_rel_res=i.true_rel_res,
                 x0_scale=i.x0_scale) for i in info]


def pcg_solve_batched(problems, fs, us, nrhs=None, rtol: float = 1e-8, maxit: int = 200, x0_given: bool = False,
                      precision=FP64, stream=None, check=True, graph: bool = False):
    """stfd_pcg_solve_batched: job k solves problems[k] for nrhs[k] stacked systems fs[k] -> us[k]."""
    count = len(problems)
    nrhs = list(nrhs) if nrhs is not None else [1] * count
    precision = PRECISIONS.get(precision, precision)
    handles = (_VP * count)(*[pr._h.value for pr in problems])
    fp = (_VP * count)(*[_dev_ptr(f, pr.N * n, "f").value for pr, f, n in zip(problems, fs, nrhs)])
    up = (_VP * count)(*[_dev_ptr(u, pr.N * n, "u").value for pr, u, n in zip(problems, us, nrhs)])
    nr = (_I64 * count)(*nrhs)
    info = (PcgInfo * sum(nrhs))()
    flags = (X0_GIVEN if x0_given else X0_ZERO) | (PCG_GRAPH if graph else 0)
    rc = _lib().stfd_pcg_solve_batched(handles, count, fp, up, nr, rtol, maxit, flags, precision, info,
                                       _stream_ptr(stream))
    if check:
        _check(rc, "stfd_pcg_solve_batched", allow=(OK, NOT_CONVERGED))
    return rc, _infos(info)


def debug_mfma_layout():
    o64 = np.empty(256)
    o32 = np.empty(256, dtype=np.float32)
    obf = np.empty(256, dtype=np.float32)
    _check(_lib().stfd_debug_mfma_layout(_dptr(o64), o32.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         obf.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
           "stfd_debug_mfma_layout")
    return o64, o32, obf


def _dev_ptr_f32(t, n_expected, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if t.numel() != n_expected:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n_expected}")
    return ctypes.c_void_p(t.data_ptr())


class Fno:
    """Handle of the spectral-convolution network (include/stfd_fno.h)."""

    def __init__(self, H, W, c_in, width=32, modes1=16, modes2=16, layers=4, proj=128, c_out=1, max_batch=1,
                 seed=0):
        self.desc = FnoDesc(H, W, c_in, width, modes1, modes2, layers, proj, c_out, max_batch, seed)
        h = ctypes.c_void_p()
        self._h = None
        _check(_lib().stfd_fno_create(ctypes.byref(self.desc), ctypes.byref(h)), "stfd_fno_create")
        self._h = h
        n = ctypes.c_int64()
        _check(_lib().stfd_fno_num_params(self._h, ctypes.byref(n)), "stfd_fno_num_params")
        self.n_params = n.value
        self.n_in = H * W * c_in
        self.n_out = H * W * c_out

    def close(self):
        if self._h is not None and _LIB is not None:
            _LIB.stfd_fno_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(_lib().stfd_fno_get_params(self._h, out.ctypes.data_as(_FP)), "stfd_fno_get_params")
        return out

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != self.n_params:
            raise ValueError("wrong parameter count")
        _check(_lib().stfd_fno_set_params(self._h, th.ctypes.data_as(_FP)), "stfd_fno_set_params")

    def get_grads(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(_lib().stfd_fno_get_grads(self._h, out.ctypes.data_as(_FP)), "stfd_fno_get_grads")
        return out

    def forward(self, x, y, batch, stream=None):
        _check(_lib().stfd_fno_forward(self._h, _dev_ptr_f32(x, self.n_in * batch, "x"),
                                       _dev_ptr_f32(y, self.n_out * batch, "y"), batch, _stream_ptr(stream)),
               "stfd_fno_forward")

    def backward(self, dy, batch, dx=None, stream=None):
        _check(_lib().stfd_fno_backward(self._h, _dev_ptr_f32(dy, self.n_out * batch, "dy"),
                                        _dev_ptr_f32(dx, self.n_in * batch, "dx") if dx is not None else None,
                                        batch, _stream_ptr(stream)), "stfd_fno_backward")

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib().stfd_fno_adam_step(self._h, lr, beta1, beta2, eps, _stream_ptr(stream)), "stfd_fno_adam_step")


def fno_rel_l2(y, t, n, batch, dy=None, stream=None):
    """stfd_fno_rel_l2: mean relative l2 error over `batch` samples of n values; fills dy if given."""
    loss = ctypes.c_float()
    _check(_lib().stfd_fno_rel_l2(_dev_ptr_f32(y, n * batch, "y"), _dev_ptr_f32(t, n * batch, "t"), n, batch,
                                  _dev_ptr_f32(dy, n * batch, "dy") if dy is not None else None,
                                  ctypes.byref(loss), _stream_ptr(stream)), "stfd_fno_rel_l2")
    return loss.value


def fno_to_f64(y, x, n, stream=None):
    """stfd_fno_to_f64: FP32 network output -> FP64 (complex128 tensor x of n / 2 entries)."""
    _check(_lib().stfd_fno_to_f64(_dev_ptr_f32(y, n, "y"), _dev_ptr(x, n // 2, "x"), n, _stream_ptr(stream)),
           "stfd_fno_to_f64")


def fno_diff_f64(y, t, e, stream=None):
    """stfd_fno_diff_f64: e (complex128 tensor) = y - t (float32 tensors of 2 e.numel() values; t may be None)."""
    n = 2 * e.numel()
    _check(_lib().stfd_fno_diff_f64(_dev_ptr_f32(y, n, "y"), _dev_ptr_f32(t, n, "t") if t is not None else None,
                                    _dev_ptr(e, n // 2, "e"), n, _stream_ptr(stream)), "stfd_fno_diff_f64")


def fno_energy_loss(e, Ae, n, batch, t_energy=None, dy=None, stream=None):
    """stfd_fno_energy_loss: returns (loss, per-sample energies e^H A e); fills dy if given."""
    import torch
    loss = ctypes.c_float()
    en = np.empty(batch, dtype=np.float64)
    if t_energy is not None and not (t_energy.is_cuda and t_energy.dtype == torch.float64 and t_energy.numel() == batch):
        raise ValueError("t_energy must be a float64 CUDA tensor with one entry per sample")
    _check(_lib().stfd_fno_energy_loss(_dev_ptr(e, n // 2 * batch, "e"), _dev_ptr(Ae, n // 2 * batch, "Ae"),
                                       ctypes.c_void_p(t_energy.data_ptr()) if t_energy is not None else None, n,
                                       batch, _dev_ptr_f32(dy, n * batch, "dy") if dy is not None else None,
                                       en.ctypes.data_as(_DP), ctypes.byref(loss), _stream_ptr(stream)),
           "stfd_fno_energy_loss")
    return loss.value, en
