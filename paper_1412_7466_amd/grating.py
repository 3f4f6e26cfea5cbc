"""Thin ctypes binding of libgrating.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts a
``paper_1412_7466_amd.inputs.Problem`` into the C structs of include/grating.h,
allocates device vectors with torch, and passes pointers and the stream.  It
raises if the library is missing: there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrating.so")

GRT_OK, GRT_EINVAL, GRT_EGEOM, GRT_ENOMEM, GRT_EHIP, GRT_ENOCONV, GRT_ESTATE, GRT_EUNSUP = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "GRT_OK", -1: "GRT_EINVAL", -2: "GRT_EGEOM", -3: "GRT_ENOMEM", -4: "GRT_EHIP",
                -5: "GRT_ENOCONV", -6: "GRT_ESTATE", -7: "GRT_EUNSUP"}
GRT_FP64, GRT_FP32, GRT_FP32_RELAXED = 0, 1, 2
GRT_TM, GRT_TE = 0, 1


class grt_layers(C.Structure):
    _fields_ = [("d", C.c_double), ("h", C.c_double), ("y0", C.c_double),
                ("n_layer", C.c_double * 3), ("N", C.c_int), ("Nw", C.c_int * 3),
                ("Q", C.c_int * 3), ("Nu", C.c_int), ("n_rb_lo", C.c_int), ("Nrb", C.c_int),
                ("zeta_K", C.c_int), ("pinv_eps", C.c_double),
                ("n_fourier", C.c_int), ("iface", C.POINTER(C.c_double)),
                ("n3_im", C.c_double)]


class grt_inclusions(C.Structure):
    _fields_ = [("M", C.c_int64), ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("radius", C.POINTER(C.c_double)), ("n_incl", C.POINTER(C.c_double)),
                ("shape", C.POINTER(C.c_double)), ("shape_nodes", C.c_int),
                ("n_incl_im", C.POINTER(C.c_double))]


class grt_incidence(C.Structure):
    _fields_ = [("omega", C.c_double), ("phi", C.c_double), ("P", C.c_int),
                ("n_rhs", C.c_int64), ("phis", C.POINTER(C.c_double)),
                ("polarization", C.c_int)]


class grt_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("restart", C.c_int),
                ("use_x0", C.c_int), ("precision", C.c_int), ("inner_tol", C.c_double),
                ("max_refine", C.c_int), ("use_graph", C.c_int)]


class grt_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("rel_resid", C.c_double),
                ("seconds", C.c_double), ("refine_steps", C.c_int), ("x0_rejected", C.c_int),
                ("fp32_applies", C.c_int)]


class grt_sizes(C.Structure):
    _fields_ = [("M", C.c_int64), ("P", C.c_int), ("n_beta", C.c_int64), ("n_rows", C.c_int64),
                ("n_alpha", C.c_int64), ("rank", C.c_int64), ("Nrb", C.c_int),
                ("m2l_chunks", C.c_int), ("m2l_split", C.c_int), ("cx_chunks", C.c_int),
                ("bx_chunks", C.c_int), ("n_rhs", C.c_int64)]


class grt_nn_config(C.Structure):
    _fields_ = [("width", C.c_int), ("layers", C.c_int), ("k", C.c_int), ("p_out", C.c_int)]


# name -> (restype, argtypes); mirrors include/grating.h
_VP = C.c_void_p
_PROTOS = {
    "grt_create": (C.c_int, [C.POINTER(_VP), C.c_int, _VP]),
    "grt_destroy": (C.c_int, [_VP]),
    "grt_error_message": (C.c_char_p, [_VP]),
    "grt_set_problem": (C.c_int, [_VP, C.POINTER(grt_layers), C.POINTER(grt_inclusions),
                                  C.POINTER(grt_incidence)]),
    "grt_build": (C.c_int, [_VP]),
    "grt_build_translation": (C.c_int, [_VP]),
    "grt_query": (C.c_int, [_VP, C.POINTER(grt_sizes)]),
    "grt_apply": (C.c_int, [_VP, _VP, _VP, C.c_int]),
    "grt_apply_T": (C.c_int, [_VP, _VP, _VP]),
    "grt_apply_ST_block": (C.c_int, [_VP, _VP, _VP]),
    "grt_apply_lowrank": (C.c_int, [_VP, _VP, _VP]),
    "grt_rhs": (C.c_int, [_VP, _VP]),
    "grt_incident": (C.c_int, [_VP, _VP]),
    "grt_set_table": (C.c_int, [_VP, C.c_int]),
    "grt_set_table32": (C.c_int, [_VP, C.c_int]),
    "grt_scattering_blocks": (C.c_int, [_VP, _VP]),
    "grt_table_bytes": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "grt_set_launch": (C.c_int, [_VP, C.c_int, C.c_int]),
    "grt_set_overlap": (C.c_int, [_VP, C.c_int]),
    "grt_set_fmm": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "grt_autotune": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "grt_solve": (C.c_int, [_VP, C.POINTER(grt_solve_opts), _VP, C.POINTER(grt_solve_stats)]),
    "grt_bragg": (C.c_int, [_VP, C.c_int64, _VP, C.c_int64, C.POINTER(C.c_int), C.POINTER(C.c_double),
                            C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                            C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "grt_eval_field": (C.c_int, [_VP, C.c_int64, _VP, C.c_int64, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]),
    "grt_get_A": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "grt_get_mie": (C.c_int, [_VP, C.POINTER(C.c_double)]),
    "grt_profile_enable": (C.c_int, [_VP, C.c_int]),
    "grt_profile_read": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "grt_apply_T_noalloc": (C.c_int, [C.c_int64, C.c_int, C.c_double, C.c_double, C.c_double,
                                      C.c_double, _VP, _VP, _VP, _VP, _VP]),
    "grt_batch_create": (C.c_int, [C.POINTER(_VP), C.c_int64, C.POINTER(_VP), _VP]),
    "grt_batch_destroy": (C.c_int, [_VP]),
    "grt_batch_error_message": (C.c_char_p, [_VP]),
    "grt_batch_solve": (C.c_int, [_VP, C.POINTER(grt_solve_opts), C.POINTER(_VP),
                                  C.POINTER(grt_solve_stats)]),
    "grt_nn_create": (C.c_int, [C.POINTER(_VP), C.c_int, _VP, C.POINTER(grt_nn_config)]),
    "grt_nn_destroy": (C.c_int, [_VP]),
    "grt_nn_error_message": (C.c_char_p, [_VP]),
    "grt_nn_num_params": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "grt_nn_set_params": (C.c_int, [_VP, C.POINTER(C.c_float), C.c_int64]),
    "grt_nn_get_params": (C.c_int, [_VP, C.POINTER(C.c_float), C.c_int64]),
    "grt_nn_add_sample": (C.c_int, [_VP, _VP, _VP, C.POINTER(C.c_int)]),
    "grt_nn_clear_samples": (C.c_int, [_VP]),
    "grt_nn_sample_size": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_int64)]),
    "grt_nn_get_sample": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_int),
                                    C.POINTER(C.c_float), C.POINTER(C.c_float),
                                    C.POINTER(C.c_float), C.POINTER(C.c_double)]),
    "grt_nn_set_target": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                    C.c_double]),
    "grt_nn_loss_grad": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_float),
                                   C.POINTER(C.c_float)]),
    "grt_nn_train": (C.c_int, [_VP, C.c_int64, C.POINTER(C.c_int), C.c_int, C.c_float,
                               C.c_uint64, C.POINTER(C.c_double)]),
    "grt_nn_predict": (C.c_int, [_VP, _VP, _VP]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgrating.so and declare every prototype; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime: load it first so that this library binds to
    # the same one (streams and device memory are shared with torch).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built: run `python -m paper_1412_7466_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GratingError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Context:
    """One problem on one GPU.  Vectors are torch complex128 tensors on the device."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        h = _VP()
        st = self.lib.grt_create(C.byref(h), device, _VP(self.stream.cuda_stream))
        if st != GRT_OK:
            raise GratingError(st, "grt_create failed")
        self.h = h
        self.sizes = None

    # -- plumbing ------------------------------------------------------------
    def _check(self, st):
        if st != GRT_OK:
            msg = self.lib.grt_error_message(self.h)
            raise GratingError(st, msg.decode() if msg else "")

    def _enter(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _leave(self):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.grt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- problem ---------------------------------------------------------------
    def set_problem(self, pb, phis=None):
        """phis: several incidence angles (right-hand sides) on this geometry; vectors
        are then [len(phis)][M][2P+1] (flat)."""
        dd = pb.disc
        lay = grt_layers(d=pb.d, h=pb.h, y0=dd.y0, n_layer=(C.c_double * 3)(*pb.n_layer),
                         N=dd.N, Nw=(C.c_int * 3)(*dd.Nw), Q=(C.c_int * 3)(*dd.Q), Nu=dd.Nu,
                         n_rb_lo=dd.n_rb_lo, Nrb=dd.Nrb, zeta_K=dd.zeta_K,
                         pinv_eps=dd.pinv_eps, n3_im=float(getattr(pb, "n3_im", 0.0) or 0.0))
        iface = getattr(pb, "interface", None)
        if iface is not None:
            self._iface = np.ascontiguousarray(iface, dtype=np.float64).reshape(2, 2, -1)
            lay.n_fourier = self._iface.shape[2]
            lay.iface = _dptr(self._iface)
        self._arrs = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (pb.x, pb.y, pb.radius, pb.n_incl)]
        inc = grt_inclusions(M=pb.M, x=_dptr(self._arrs[0]), y=_dptr(self._arrs[1]),
                             radius=_dptr(self._arrs[2]), n_incl=_dptr(self._arrs[3]))
        shape = getattr(pb, "shape", None)
        if shape is not None:
            self._arrs.append(np.ascontiguousarray(shape, dtype=np.float64).reshape(-1))
            inc.shape = _dptr(self._arrs[4])
            inc.shape_nodes = int(pb.shape_nodes)
        n_im = getattr(pb, "n_incl_im", None)
        if n_im is not None:
            self._n_im = np.ascontiguousarray(n_im, dtype=np.float64)
            inc.n_incl_im = _dptr(self._n_im)
        pol = GRT_TE if getattr(pb, "polarization", "TM") == "TE" else GRT_TM
        if phis is not None and len(phis) > 1:
            self._phis = np.ascontiguousarray(phis, dtype=np.float64)
            wave = grt_incidence(omega=pb.omega, phi=float(self._phis[0]), P=pb.P,
                                 n_rhs=len(self._phis), phis=_dptr(self._phis), polarization=pol)
        else:
            wave = grt_incidence(omega=pb.omega, phi=pb.phi if phis is None else float(phis[0]),
                                 P=pb.P, n_rhs=0, phis=None, polarization=pol)
        self._check(self.lib.grt_set_problem(self.h, C.byref(lay), C.byref(inc), C.byref(wave)))
        self.pb = pb
        self.sizes = self.query()

    def build(self):
        self._enter()
        self._check(self.lib.grt_build(self.h))
        self._leave()
        self.sizes = self.query()

    def build_translation(self):
        """Translation data only (no layered structure): apply_ST_block, apply_T."""
        self._enter()
        self._check(self.lib.grt_build_translation(self.h))
        self._leave()
        self.sizes = self.query()

    def query(self):
        s = grt_sizes()
        self._check(self.lib.grt_query(self.h, C.byref(s)))
        return s

    @property
    def n_rhs(self):
        return max(1, int(self.sizes.n_rhs))

    def new_vec(self, one=False):
        """Zero vector of every right-hand side ([n_rhs][n_beta] flat), or of one."""
        n = int(self.sizes.n_beta) * (1 if one else self.n_rhs)
        return self.torch.zeros(n, dtype=self.torch.complex128, device=f"cuda:{self.device}")

    def _vec_ptr(self, t, one=False):
        n = int(self.sizes.n_beta) * (1 if one else self.n_rhs)
        if t.dtype != self.torch.complex128 or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"expected a contiguous complex128 vector of length {n}")
        return _VP(t.data_ptr())

    # -- operator --------------------------------------------------------------
    def apply(self, x, y=None, precision=GRT_FP64):
        y = self.new_vec() if y is None else y
        self._enter()
        self._check(self.lib.grt_apply(self.h, self._vec_ptr(x), self._vec_ptr(y), precision))
        self._leave()
        return y

    def apply_T(self, x, y=None):
        y = self.new_vec() if y is None else y
        self._enter()
        self._check(self.lib.grt_apply_T(self.h, self._vec_ptr(x), self._vec_ptr(y)))
        self._leave()
        return y

    def apply_ST_block(self, x, y=None):
        """y_r = S T_r x_r on the FP32 matrix cores for every right-hand side."""
        y = self.new_vec() if y is None else y
        self._enter()
        self._check(self.lib.grt_apply_ST_block(self.h, self._vec_ptr(x), self._vec_ptr(y)))
        self._leave()
        return y

    def apply_lowrank(self, x, y=None):
        y = self.new_vec() if y is None else y
        self._enter()
        self._check(self.lib.grt_apply_lowrank(self.h, self._vec_ptr(x), self._vec_ptr(y)))
        self._leave()
        return y

    def rhs(self, b=None):
        b = self.new_vec() if b is None else b
        self._enter()
        self._check(self.lib.grt_rhs(self.h, self._vec_ptr(b)))
        self._leave()
        return b

    def set_table(self, mode=1):
        """Resident translation table of the FP64 apply: 0 off (generator on the
        fly), 1 on (one lane per target), 2 on (two lanes per target)."""
        self._enter()
        self._check(self.lib.grt_set_table(self.h, int(mode)))
        self._leave()

    def scattering_blocks(self):
        """The block-diagonal scattering matrix, [M][2P+1][2P+1] complex (device)."""
        nb = 2 * self.pb.P + 1
        out = self.torch.zeros((self.pb.M, nb, nb), dtype=self.torch.complex128,
                               device=f"cuda:{self.device}")
        self._enter()
        self._check(self.lib.grt_scattering_blocks(self.h, _VP(out.data_ptr())))
        self._leave()
        return out

    def set_table32(self, on=True):
        """Resident FP32 table of the well-separated pairs for the mixed-precision
        apply (GRT_FP32 / GRT_FP32_RELAXED solves); False frees it."""
        self._enter()
        self._check(self.lib.grt_set_table32(self.h, int(bool(on))))
        self._leave()

    def set_launch(self, m2l_chunks, m2l_split=1):
        """Translation launch shape by hand: about m2l_chunks source chunks, split 1
        or 2 (two launches, half of the outputs each)."""
        self._enter()
        self._check(self.lib.grt_set_launch(self.h, int(m2l_chunks), int(m2l_split)))
        self._leave()
        self.sizes = self.query()

    def set_overlap(self, on):
        """Run C x, A^+ and B_phys w on a second stream, concurrently with T x."""
        self._enter()
        self._check(self.lib.grt_set_overlap(self.h, int(bool(on))))
        self._leave()

    def set_fmm(self, on=True, p_cell=0, per_cell=0):
        """Fast cell translation for large M (on) or the dense one (off); returns
        (nx, ny, p) of the cell grid."""
        info = (C.c_int * 3)()
        self._enter()
        self._check(self.lib.grt_set_fmm(self.h, int(bool(on)), int(p_cell), int(per_cell), info))
        self._leave()
        return tuple(info[:])

    def autotune(self, cap=32):
        """Time the translation launch for several chunk counts (and, on the fly,
        split over two launches or not) and keep the fastest, then the same for the
        C x and B_phys w launches; returns the translation's [(chunks, split, ms per
        launch)] (the choices are in self.sizes)."""
        n = C.c_int(0)
        ch = (C.c_int * cap)()
        sp = (C.c_int * cap)()
        ms = (C.c_double * cap)()
        self._enter()
        self._check(self.lib.grt_autotune(self.h, cap, C.byref(n), ch, sp, ms))
        self._leave()
        self.sizes = self.query()
        return [(ch[i], sp[i], ms[i]) for i in range(n.value)]

    def table_bytes(self):
        n = C.c_int64(0)
        self._check(self.lib.grt_table_bytes(self.h, C.byref(n)))
        return n.value

    def incident(self, a=None):
        """alpha0 = B_phys A^+ f (the layers' incoming coefficients at each inclusion)."""
        a = self.new_vec() if a is None else a
        self._enter()
        self._check(self.lib.grt_incident(self.h, self._vec_ptr(a)))
        self._leave()
        return a

    def solve(self, tol=1e-9, maxit=1000, restart=200, x0=None, out=None, check=True,
              precision=GRT_FP64, inner_tol=0.0, max_refine=10, graph=False):
        """GMRES to tol (FP64 residual).  precision GRT_FP32: FP64 refinement around
        inner solves on the mixed operator (inner_tol 0: 1e-5); GRT_FP32_RELAXED: one
        FP64 GMRES whose applies switch to the mixed operator below inner_tol (0:
        1e5 tol, at most 1e-2).  Returns (beta, stats) (lists of stats with several
        angles)."""
        beta = self.new_vec() if out is None else out
        if x0 is not None:
            beta.copy_(x0)
        opts = grt_solve_opts(tol=tol, maxit=maxit, restart=restart, use_x0=int(x0 is not None),
                              precision=precision, inner_tol=inner_tol, max_refine=max_refine,
                              use_graph=int(graph))
        R = self.n_rhs
        stats = (grt_solve_stats * R)()
        self._enter()
        st = self.lib.grt_solve(self.h, C.byref(opts), self._vec_ptr(beta), stats)
        self._leave()
        if check or st != GRT_ENOCONV:
            self._check(st)
        return beta, (stats[0] if R == 1 else list(stats))

    def bragg(self, beta=None, rhs=0):
        """Bragg amplitudes of right-hand side rhs; beta: that angle's vector [n_beta]."""
        n = int(self.sizes.Nrb)
        orders = (C.c_int * n)()
        c = np.zeros(2 * n)
        d = np.zeros(2 * n)
        R = np.zeros(n)
        T = np.zeros(n)
        flux = C.c_double(0)
        absorbed = C.c_double(0)
        bp = self._vec_ptr(beta, one=True) if beta is not None else _VP(0)
        self._enter()
        self._check(self.lib.grt_bragg(self.h, rhs, bp, n, orders, _dptr(c), _dptr(d), _dptr(R),
                                       _dptr(T), C.byref(flux), C.byref(absorbed)))
        self._leave()
        return dict(orders=np.array(orders[:]), c=c[0::2] + 1j * c[1::2], d=d[0::2] + 1j * d[1::2],
                    R=R, T=T, flux_err=flux.value, absorbed=absorbed.value)

    def eval_field(self, beta, xy, rhs=0):
        """Total field at the points xy ([n, 2] float64, host) for the solution beta
        (device tensor, or None without inclusions): complex128 numpy array [n]."""
        import numpy as np
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        out = np.zeros(2 * len(xy))
        self._enter()
        self._check(self.lib.grt_eval_field(self.h, rhs, self._vec_ptr(beta, one=True) if beta is not None
                                            else None, len(xy), _dptr(xy), _dptr(out)))
        self._leave()
        return out[0::2] + 1j * out[1::2]

    def get_A(self):
        s = self.sizes
        A = np.zeros(2 * s.n_rows * s.n_alpha)
        E = np.zeros(s.n_alpha)
        self._check(self.lib.grt_get_A(self.h, _dptr(A), _dptr(E)))
        A = (A[0::2] + 1j * A[1::2]).reshape(s.n_alpha, s.n_rows).T
        return A, E

    def profile(self, enable=True):
        self._check(self.lib.grt_profile_enable(self.h, int(enable)))

    def profile_read(self):
        """(total ms, launches) of the translation kernel since the last read."""
        ms = C.c_double(0)
        n = C.c_int64(0)
        self._check(self.lib.grt_profile_read(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def get_mie(self):
        s = np.zeros(2 * self.sizes.n_beta)
        self._check(self.lib.grt_get_mie(self.h, _dptr(s)))
        return s[0::2] + 1j * s[1::2]


def apply_T_noalloc(P, k2, d, alpha, cx, cy, x, y):
    """y = T x through grt_apply_T_noalloc (no context, no allocation by the call).

    cx, cy: float64 device tensors [M]; x, y: complex128 device tensors [M (2P+1)],
    all contiguous on the current device; alpha: complex Bloch phase.  Enqueued on
    torch's current stream."""
    import torch
    lib = load_library()
    M = cx.numel()
    for t in (cx, cy, x, y):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("device tensors must be contiguous CUDA tensors")
    if cy.numel() != M or x.numel() != M * (2 * P + 1) or y.numel() != x.numel():
        raise ValueError("sizes do not match M and P")
    s = torch.cuda.current_stream(x.device).cuda_stream
    st = lib.grt_apply_T_noalloc(M, P, float(k2), float(d), float(alpha.real),
                                 float(alpha.imag), _VP(cx.data_ptr()), _VP(cy.data_ptr()),
                                 _VP(x.data_ptr()), _VP(y.data_ptr()), _VP(s))
    if st != GRT_OK:
        raise GratingError(st, "grt_apply_T_noalloc failed")
    return y


class Batch:
    """Lockstep FP64 solves of several built contexts on one GPU (grt_batch_*).

    The contexts must stay alive and untouched while the batch exists."""

    def __init__(self, contexts):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.ctxs = list(contexts)
        if not self.ctxs:
            raise ValueError("empty batch")
        self.device = self.ctxs[0].device
        self.stream = torch.cuda.Stream(device=self.device)
        arr = (_VP * len(self.ctxs))(*[c.h for c in self.ctxs])
        h = _VP()
        st = self.lib.grt_batch_create(C.byref(h), len(self.ctxs), arr,
                                       _VP(self.stream.cuda_stream))
        if st != GRT_OK:
            raise GratingError(st, "grt_batch_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.grt_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, tol=1e-9, maxit=1000, restart=200, x0=None, check=True, graph=False,
              precision=None, inner_tol=0.0, max_refine=0):
        """Returns (list of beta vectors, list of grt_solve_stats).  precision
        GRT_FP32: FP32 translation inside lockstep FP64 refinement."""
        betas = [c.new_vec() for c in self.ctxs]
        if x0 is not None:
            for b, x in zip(betas, x0):
                b.copy_(x)
        ptrs = (_VP * len(betas))(*[c._vec_ptr(b) for c, b in zip(self.ctxs, betas)])
        opts = grt_solve_opts(tol=tol, maxit=maxit, restart=restart, use_x0=int(x0 is not None),
                              precision=GRT_FP64 if precision is None else precision,
                              inner_tol=inner_tol, max_refine=max_refine, use_graph=int(graph))
        stats = (grt_solve_stats * len(betas))()
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        st = self.lib.grt_batch_solve(self.h, C.byref(opts), ptrs, stats)
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        if st != GRT_OK and (check or st != GRT_ENOCONV):
            msg = self.lib.grt_batch_error_message(self.h)
            raise GratingError(st, msg.decode() if msg else "")
        return betas, list(stats)


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Network:
    """The learned warm start (grt_nn_*): a message-passing network on one GPU."""

    def __init__(self, width=128, layers=3, k=16, p_out=3, device=0):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = device
        self.width, self.layers, self.k, self.p_out = width, layers, k, p_out
        self.O = 2 * (2 * p_out + 1)
        self.stream = torch.cuda.Stream(device=device)
        cfg = grt_nn_config(width=width, layers=layers, k=k, p_out=p_out)
        h = _VP()
        st = self.lib.grt_nn_create(C.byref(h), device, _VP(self.stream.cuda_stream), C.byref(cfg))
        if st != GRT_OK:
            raise GratingError(st, "grt_nn_create failed")
        self.h = h
        n = C.c_int64(0)
        self._check(self.lib.grt_nn_num_params(self.h, C.byref(n)))
        self.n_params = n.value

    def _check(self, st):
        if st != GRT_OK:
            msg = self.lib.grt_nn_error_message(self.h)
            raise GratingError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.grt_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        self._check(self.lib.grt_nn_set_params(self.h, _fptr(a), a.size))

    def get_params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.lib.grt_nn_get_params(self.h, _fptr(a), a.size))
        return a

    def add_sample(self, ctx, beta=None):
        i = C.c_int(0)
        ctx.torch.cuda.synchronize(self.device)
        bp = ctx._vec_ptr(beta) if beta is not None else _VP(0)
        self._check(self.lib.grt_nn_add_sample(self.h, ctx.h, bp, C.byref(i)))
        return i.value

    def clear_samples(self):
        self._check(self.lib.grt_nn_clear_samples(self.h))

    def sample(self, i):
        M = C.c_int64(0)
        self._check(self.lib.grt_nn_sample_size(self.h, i, C.byref(M)))
        M = M.value
        feat = np.zeros((M, 32), np.float32)
        nbr = np.zeros((M, self.k), np.int32)
        edge = np.zeros((M, self.k, 8), np.float32)
        t = np.zeros((M, self.O), np.float32)
        w = np.zeros((M, self.O), np.float32)
        wn = C.c_double(0)
        self._check(self.lib.grt_nn_get_sample(
            self.h, i, _fptr(feat), nbr.ctypes.data_as(C.POINTER(C.c_int)), _fptr(edge),
            _fptr(t), _fptr(w), C.byref(wn)))
        return dict(feat=feat, nbr=nbr, edge=edge, target=t, weight=w, wnorm=wn.value)

    def set_target(self, i, t, w, wnorm):
        t = np.ascontiguousarray(t, dtype=np.float32)
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self.lib.grt_nn_set_target(self.h, i, _fptr(t), _fptr(w), float(wnorm)))

    def loss_grad(self, i):
        M = C.c_int64(0)
        self._check(self.lib.grt_nn_sample_size(self.h, i, C.byref(M)))
        loss = C.c_double(0)
        g = np.zeros(self.n_params, np.float32)
        out = np.zeros((M.value, self.O), np.float32)
        self._check(self.lib.grt_nn_loss_grad(self.h, i, C.byref(loss), _fptr(g), _fptr(out)))
        return loss.value, g, out

    def train(self, ids, epochs=1, lr=1e-3, seed=0):
        a = (C.c_int * len(ids))(*ids)
        loss = C.c_double(0)
        self._check(self.lib.grt_nn_train(self.h, len(ids), a, epochs, lr, seed, C.byref(loss)))
        return loss.value

    def predict(self, ctx, out=None):
        beta0 = ctx.new_vec() if out is None else out
        ctx.torch.cuda.synchronize(self.device)
        self._check(self.lib.grt_nn_predict(self.h, ctx.h, ctx._vec_ptr(beta0)))
        return beta0


def exported_symbols():
    """Names declared in include/grating.h (parsed from the header text)."""
    import re
    hdr = os.path.join(_HERE, "..", "include", "grating.h")
    txt = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:grt_status|const char\s*\*)\s*(grt_\w+)\s*\(", txt, re.M)))
