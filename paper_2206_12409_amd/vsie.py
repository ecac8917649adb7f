"""ctypes binding of libvsie.so (the C ABI declared in include/vsie.h).

Argument marshalling only: every step of setup, matrix-vector product and solve runs in the
library. torch supplies device memory and the HIP stream. If the library is not built the
binding raises; there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvsie.so")

VSIE_OK, VSIE_E_NOCONV = 0, 7
VSIE_NEAR, VSIE_FAR = 0, 1
VSIE_C128, VSIE_C64 = 0, 1
VSIE_GMRES64, VSIE_IR_MIXED, VSIE_SCHUR, VSIE_SCHUR_MIXED, VSIE_SCHUR_LEARNED = 0, 1, 2, 3, 4
VSIE_E_SINGULAR = 11
VSIE_E_UNSUPPORTED = 9
VSIE_BASIS_PWC, VSIE_BASIS_PWL = 0, 1
VSIE_PREC_FP64, VSIE_PREC_MIXED = 0, 1
X_TT_CORES, X_ACA, X_STENCIL, X_GENERATOR, X_EXT_GRID = 1, 2, 3, 4, 5

EXPORTED = ["vsie_default_options", "vsie_default_solve_opts", "vsie_create", "vsie_create_shared", "vsie_sizes",
            "vsie_rhs", "vsie_graph_create", "vsie_graph_launch", "vsie_graph_destroy",
            "vsie_matvec", "vsie_matvec_graph", "vsie_zpass_tuning", "vsie_zpass_select", "vsie_solve", "vsie_solve_ports", "vsie_port_current", "vsie_export", "vsie_import",
            "vsie_checkpoint_save", "vsie_checkpoint_load", "vsie_set_concurrency",
            "vsie_profile", "vsie_profile_mask", "vsie_profile_read", "vsie_schur_setup", "vsie_schur_info",
            "vsie_schur_matvec", "vsie_schur_precond", "vsie_dense_lu_solve", "vsie_dense_lu_solve_noalloc",
            "vsie_net_create", "vsie_net_destroy", "vsie_net_info", "vsie_net_get_params", "vsie_net_set_params",
            "vsie_net_collect", "vsie_net_train", "vsie_net_attach", "vsie_net_forward", "vsie_net_gradients",
            "vsie_net_adam", "vsie_net_layer", "vsie_net_layer_wgrad", "vsie_destroy", "vsie_last_error"]


STAGES = ["build_grid", "fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv", "body_out", "pfft_gather",
          "gemv_far", "precorrect", "aca", "tt_pre", "gemv_far_reduce", "tt_post"]


class Mesh(C.Structure):
    _fields_ = [("verts", C.POINTER(C.c_double)), ("n_verts", C.c_int32), ("tris", C.POINTER(C.c_int32)),
                ("n_tris", C.c_int32), ("domain", C.c_int32), ("port_edges", C.POINTER(C.c_int32)),
                ("port_id", C.POINTER(C.c_int32)), ("n_port_edges", C.c_int32)]


class ProblemC(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("origin", C.c_double * 3), ("freq_hz", C.c_double),
                ("eps_r", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)), ("n_meshes", C.c_int32),
                ("meshes", C.POINTER(Mesh))]


class Options(C.Structure):
    _fields_ = [("tt_tol", C.c_double), ("tt_rank_max", C.c_int32), ("aca_tol", C.c_double),
                ("aca_rank_max", C.c_int32), ("precorrect_dist", C.c_int32), ("precision", C.c_int32),
                ("build_far", C.c_int32), ("seed", C.c_uint64), ("basis", C.c_int32), ("stencil", C.c_int32),
                ("quad_near_vol", C.c_int32), ("quad_near_surf", C.c_int32), ("quad_far_vol", C.c_int32),
                ("quad_far_surf", C.c_int32)]


class Sizes(C.Structure):
    _fields_ = [("n_total", C.c_int64), ("m_far", C.c_int32), ("m_near", C.c_int32), ("n", C.c_int32 * 3),
                ("n_ext", C.c_int32 * 3), ("fft", C.c_int32 * 3), ("n_ports", C.c_int32), ("n_tissue", C.c_int32),
                ("tt_rank", (C.c_int32 * 3) * 3), ("tt_err_est", C.c_double * 3), ("aca_rank", C.c_int32),
                ("precorr_nnz", C.c_int64), ("device_bytes", C.c_int64), ("setup_seconds", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32), ("method", C.c_int32),
                ("inner_tol", C.c_double), ("precond", C.c_int32), ("reorth", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("refinements", C.c_int32),
                ("rel_residual", C.c_double), ("block_residual", C.c_double * 3), ("seconds", C.c_double),
                ("gs_second_passes", C.c_int32)]


_lib = None


def load(path=LIB_PATH):
    """Load libvsie.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libvsie.so is not built: run paper_2206_12409_amd.build.build()")
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.vsie_default_options.argtypes = [C.POINTER(Options)]
    lib.vsie_default_solve_opts.argtypes = [C.POINTER(SolveOpts)]
    lib.vsie_create.argtypes = [C.POINTER(ProblemC), C.POINTER(Options), vp, C.POINTER(vp)]
    lib.vsie_create_shared.argtypes = [C.POINTER(ProblemC), C.POINTER(Options), vp, vp, C.POINTER(vp)]
    lib.vsie_graph_create.argtypes = [C.c_int, C.POINTER(vp), C.c_int, C.POINTER(C.c_int), C.POINTER(vp),
                                      C.POINTER(vp), vp, C.POINTER(vp)]
    lib.vsie_graph_launch.argtypes = [vp, vp]
    lib.vsie_graph_destroy.argtypes = [vp]
    lib.vsie_sizes.argtypes = [vp, C.POINTER(Sizes)]
    lib.vsie_rhs.argtypes = [vp, C.c_int, C.c_int, vp, vp]
    lib.vsie_matvec.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp]
    lib.vsie_matvec_graph.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp]
    lib.vsie_zpass_tuning.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_double)]
    lib.vsie_zpass_select.argtypes = [vp, C.c_int, C.c_int]
    lib.vsie_solve.argtypes = [vp, C.POINTER(SolveOpts), C.c_int, vp, vp, C.POINTER(SolveStats), vp]
    lib.vsie_solve_ports.argtypes = [vp, C.POINTER(SolveOpts), C.c_int, C.POINTER(C.c_int32), vp,
                                     C.POINTER(SolveStats), vp]
    lib.vsie_port_current.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.vsie_export.argtypes = [vp, C.c_int, C.c_int, vp, C.POINTER(C.c_size_t)]
    lib.vsie_import.argtypes = [vp, C.c_int, C.c_int, vp, C.c_size_t]
    lib.vsie_checkpoint_save.argtypes = [vp, C.c_char_p]
    lib.vsie_checkpoint_load.argtypes = [vp, C.c_char_p]
    lib.vsie_profile.argtypes = [vp, C.c_int]
    lib.vsie_profile_mask.argtypes = [vp, C.c_uint32]
    lib.vsie_set_concurrency.argtypes = [vp, C.c_int]
    lib.vsie_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int)]
    lib.vsie_schur_setup.argtypes = [vp, C.c_int]
    lib.vsie_schur_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.vsie_schur_matvec.argtypes = [vp, vp, vp, vp]
    lib.vsie_schur_precond.argtypes = [vp, vp, vp, vp]
    lib.vsie_dense_lu_solve.argtypes = [C.c_int, vp, C.c_int64, vp, C.c_int64, C.c_int, vp]
    lib.vsie_dense_lu_solve_noalloc.argtypes = [C.c_int, vp, C.c_int64, vp, C.c_int64, C.c_int, vp]
    fp = C.POINTER(C.c_float)
    lib.vsie_net_create.argtypes = [C.c_uint64, C.c_int64, C.POINTER(vp)]
    lib.vsie_net_destroy.argtypes = [vp]
    lib.vsie_net_destroy.restype = None
    lib.vsie_net_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.vsie_net_get_params.argtypes = [vp, fp, C.c_int64]
    lib.vsie_net_set_params.argtypes = [vp, fp, C.c_int64]
    lib.vsie_net_collect.argtypes = [vp, vp, C.c_int, C.POINTER(C.c_int32), C.POINTER(SolveOpts),
                                     C.POINTER(C.c_int64), vp]
    lib.vsie_net_train.argtypes = [vp, C.c_int, C.c_float, C.c_uint64, C.POINTER(C.c_double), vp]
    lib.vsie_net_attach.argtypes = [vp, vp]
    lib.vsie_net_forward.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp]
    lib.vsie_net_gradients.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, C.POINTER(C.c_double), fp, vp]
    lib.vsie_net_adam.argtypes = [vp, C.c_float, vp]
    lib.vsie_net_layer.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp]
    lib.vsie_net_layer_wgrad.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, fp, fp, vp]
    lib.vsie_destroy.argtypes = [vp]
    lib.vsie_destroy.restype = None
    lib.vsie_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class VsieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("vsie error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != VSIE_OK:
        raise VsieError(rc, load().vsie_last_error().decode())


def default_options(**kw):
    o = Options()
    load().vsie_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    """hipStream_t of a torch stream (default: the current stream); 0 selects the null stream."""
    if isinstance(stream, int) and stream == 0:
        return C.c_void_p(None)
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Operator:
    """Hybrid VSIE operator of one problem (vsie_synth.Problem-like: grid, meshes, freq_hz)."""

    def __init__(self, problem, options=None, stream=None, share_far_with=None, **opt_kw):
        """share_far_with: an Operator over the same far conductors and frequency whose dense far
        block this one uses instead of assembling its own (vsie_create_shared)."""
        lib = load()
        g = problem.grid
        self._keep = []
        eps = np.ascontiguousarray(g.eps_r, np.float64).ravel()
        sig = np.ascontiguousarray(g.sigma, np.float64).ravel()
        self._keep += [eps, sig]
        meshes = (Mesh * max(1, len(problem.meshes)))()
        for i, m in enumerate(problem.meshes):
            v = np.ascontiguousarray(m.verts, np.float64)
            t = np.ascontiguousarray(m.tris, np.int32)
            pe = np.ascontiguousarray(m.port_edges, np.int32).reshape(-1, 2)
            pid = np.ascontiguousarray(m.port_id, np.int32)
            self._keep += [v, t, pe, pid]
            meshes[i].verts = v.ctypes.data_as(C.POINTER(C.c_double))
            meshes[i].n_verts = len(v)
            meshes[i].tris = t.ctypes.data_as(C.POINTER(C.c_int32))
            meshes[i].n_tris = len(t)
            meshes[i].domain = int(m.domain)
            meshes[i].port_edges = pe.ctypes.data_as(C.POINTER(C.c_int32))
            meshes[i].port_id = pid.ctypes.data_as(C.POINTER(C.c_int32))
            meshes[i].n_port_edges = len(pid)
        p = ProblemC()
        p.n = (C.c_int32 * 3)(*[int(x) for x in g.n])
        p.h = float(g.h)
        p.origin = (C.c_double * 3)(*[float(x) for x in g.origin])
        p.freq_hz = float(problem.freq_hz)
        p.eps_r = eps.ctypes.data_as(C.POINTER(C.c_double))
        p.sigma = sig.ctypes.data_as(C.POINTER(C.c_double))
        p.n_meshes = len(problem.meshes)
        p.meshes = meshes
        opts = options if options is not None else default_options(**opt_kw)
        h = C.c_void_p()
        if share_far_with is None:
            _check(lib.vsie_create(C.byref(p), C.byref(opts), _stream_ptr(stream), C.byref(h)))
        else:
            _check(lib.vsie_create_shared(C.byref(p), C.byref(opts), share_far_with._h, _stream_ptr(stream),
                                          C.byref(h)))
        self._h = h
        self._keep = None
        s = Sizes()
        _check(lib.vsie_sizes(self._h, C.byref(s)))
        self.sizes = s
        self.N = int(s.n_total)
        self.m_far, self.m_near = int(s.m_far), int(s.m_near)
        self.n_ports = int(s.n_ports)

    def close(self):
        if getattr(self, "_h", None):
            load().vsie_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        s = self.sizes
        return dict(N=self.N, m_far=self.m_far, m_near=self.m_near, n_ext=tuple(s.n_ext), fft=tuple(s.fft),
                    n_ports=self.n_ports, n_tissue=int(s.n_tissue),
                    tt_rank=[tuple(s.tt_rank[c]) for c in range(3)], tt_err_est=list(s.tt_err_est),
                    aca_rank=int(s.aca_rank), precorr_nnz=int(s.precorr_nnz), device_bytes=int(s.device_bytes),
                    setup_seconds=float(s.setup_seconds))

    @staticmethod
    def _dtype_code(t):
        import torch
        if t.dtype == torch.complex128:
            return VSIE_C128
        if t.dtype == torch.complex64:
            return VSIE_C64
        raise TypeError("complex128 or complex64 tensors only")

    def matvec(self, x, out=None, stream=None):
        import torch
        if x.dim() not in (1, 2) or x.shape[-1] != self.N:
            raise ValueError("x must be [N] or [nrhs][N] with N = %d, got %s" % (self.N, tuple(x.shape)))
        if not x.is_contiguous():
            raise ValueError("x must be contiguous")
        self._dtype_code(x)
        if out is not None:
            if (out.dtype != x.dtype or out.shape != x.shape or out.device != x.device
                    or not out.is_contiguous()):
                raise ValueError("out must be a contiguous tensor of x's dtype, shape and device")
            if out.data_ptr() == x.data_ptr():
                raise ValueError("out must not alias x")
        if not x.is_cuda:
            raise ValueError("x must be a device tensor")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        if nrhs < 1:
            raise ValueError("x holds no column")
        y = torch.empty_like(x) if out is None else out
        _check(load().vsie_matvec(self._h, self._dtype_code(x), nrhs, C.c_void_p(x.data_ptr()),
                                  C.c_void_p(y.data_ptr()), _stream_ptr(stream)))
        return y

    def matvec_graph(self, x, out, stream=None):
        """vsie_matvec_graph: the product replayed from a HIP graph captured for these two buffers
        (keep both tensors alive while the operator may replay it)."""
        if out is None:
            raise ValueError("the graph product needs a fixed output tensor")
        if x.dim() not in (1, 2) or x.shape[-1] != self.N or not x.is_contiguous() or not x.is_cuda:
            raise ValueError("x must be a contiguous device tensor [N] or [nrhs][N] with N = %d" % self.N)
        if (out.dtype != x.dtype or out.shape != x.shape or out.device != x.device or not out.is_contiguous()
                or out.data_ptr() == x.data_ptr()):
            raise ValueError("out must be a contiguous tensor of x's dtype, shape and device, not aliasing x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _check(load().vsie_matvec_graph(self._h, self._dtype_code(x), nrhs, C.c_void_p(x.data_ptr()),
                                        C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def zpass_tuning(self, complex64=False):
        """The setup autotuner's z-pass result: {"chosen": c, "candidates": [(v, np, ms), ...]}."""
        ch = C.c_int(0)
        v = (C.c_int * 3)()
        npb = (C.c_int * 3)()
        ms = (C.c_double * 3)()
        _check(load().vsie_zpass_tuning(self._h, VSIE_C64 if complex64 else VSIE_C128, C.byref(ch), v, npb, ms))
        return {"chosen": ch.value, "candidates": [(v[i], npb[i], ms[i]) for i in range(3)]}

    def zpass_select(self, cand, complex64=False):
        _check(load().vsie_zpass_select(self._h, VSIE_C64 if complex64 else VSIE_C128, int(cand)))

    def rhs(self, port, dtype=None, stream=None, out=None):
        """Delta-gap right-hand side of `port` (vsie_rhs), into `out` when given."""
        import torch
        dt = torch.complex128 if dtype is None else dtype
        if out is None:
            b = torch.empty(self.N, dtype=dt, device="cuda")
        else:
            if out.shape != (self.N,) or not out.is_contiguous() or not out.is_cuda:
                raise ValueError("out must be a contiguous device vector of length N")
            b = out
        _check(load().vsie_rhs(self._h, int(port), self._dtype_code(b), C.c_void_p(b.data_ptr()), _stream_ptr(stream)))
        return b

    def solve(self, b, tol=1e-6, restart=50, max_iter=5000, method=VSIE_GMRES64, inner_tol=1e-3, stream=None,
              allow_noconv=False, precond=True, reorth=0.1):
        """Solve Z x = b for each row of b (vsie_solve) from a zero start. method is VSIE_GMRES64,
        VSIE_IR_MIXED, VSIE_SCHUR or VSIE_SCHUR_MIXED; precond right-preconditions the reduced
        system of the SCHUR methods; reorth is the DGKS constant below which a Gram-Schmidt pass is
        repeated. Returns x and one stats dict per right-hand side; VSIE_E_NOCONV raises unless
        allow_noconv."""
        import torch
        if b.dim() not in (1, 2) or b.shape[-1] != self.N:
            raise ValueError("b must be [N] or [nrhs][N] with N = %d, got %s" % (self.N, tuple(b.shape)))
        if b.dtype != torch.complex128 or not b.is_contiguous():
            raise ValueError("b must be a contiguous complex128 tensor")
        if not b.is_cuda:
            raise ValueError("b must be a device tensor")
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        if nrhs < 1:
            raise ValueError("b holds no column")
        x = torch.empty_like(b)
        o = SolveOpts(tol, restart, max_iter, method, inner_tol, 1 if precond else 0, reorth)
        st = (SolveStats * nrhs)()
        rc = load().vsie_solve(self._h, C.byref(o), nrhs, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), st,
                               _stream_ptr(stream))
        if rc != VSIE_OK and not (allow_noconv and rc == VSIE_E_NOCONV):
            _check(rc)
        return x, self._stats(st, rc)

    def solve_ports(self, ports, tol=1e-6, restart=50, max_iter=5000, method=VSIE_GMRES64, inner_tol=1e-3,
                    stream=None, allow_noconv=False, precond=True, reorth=0.1):
        """Solve for the delta-gap excitation of each port in `ports` (vsie_solve_ports); returns
        x [nports][N] complex128 on the device and one stats dict per port."""
        import torch
        pl = np.ascontiguousarray([int(p) for p in ports], np.int32)
        if pl.size < 1:
            raise ValueError("no port given")
        x = torch.empty((pl.size, self.N), dtype=torch.complex128, device="cuda")
        o = SolveOpts(tol, restart, max_iter, method, inner_tol, 1 if precond else 0, reorth)
        st = (SolveStats * pl.size)()
        rc = load().vsie_solve_ports(self._h, C.byref(o), int(pl.size), pl.ctypes.data_as(C.POINTER(C.c_int32)),
                                     C.c_void_p(x.data_ptr()), st, _stream_ptr(stream))
        if rc != VSIE_OK and not (allow_noconv and rc == VSIE_E_NOCONV):
            _check(rc)
        return x, self._stats(st, rc)

    @staticmethod
    def _stats(st, rc):
        return [dict(iterations=s.iterations, restarts=s.restarts, refinements=s.refinements,
                     rel_residual=s.rel_residual, block_residual=list(s.block_residual), seconds=s.seconds,
                     gs_second_passes=s.gs_second_passes, converged=rc == VSIE_OK) for s in st]

    def schur_setup(self, precond=True):
        """Eliminate the far-conductor currents (and build the reduced system's preconditioner)."""
        _check(load().vsie_schur_setup(self._h, 1 if precond else 0))
        return self.schur_info()

    def schur_info(self):
        k = C.c_int32(0)
        sec = C.c_double(0)
        built = C.c_int32(0)
        _check(load().vsie_schur_info(self._h, C.byref(k), C.byref(sec), C.byref(built)))
        return dict(n_proxy=k.value, seconds=sec.value, eliminated=bool(built.value & 1),
                    preconditioner=bool(built.value & 2))

    def _vec_op(self, fn, x, stream):
        import torch
        if x.dtype != torch.complex128 or not x.is_cuda or not x.is_contiguous() or x.shape != (self.N,):
            raise ValueError("x must be a contiguous complex128 device vector of length N")
        y = torch.empty_like(x)
        _check(fn(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), _stream_ptr(stream)))
        return y

    def schur_matvec(self, x, stream=None):
        """Reduced operator (far currents eliminated) on the near and body parts of x."""
        return self._vec_op(load().vsie_schur_matvec, x, stream)

    def schur_precond(self, x, stream=None):
        """Block-diagonal right preconditioner of the reduced system."""
        return self._vec_op(load().vsie_schur_precond, x, stream)

    def profile(self, enable=True, stages=None):
        """Enable (and reset) or disable per-stage event timing of matvec; `stages` (names) limits
        the timing to those stages."""
        if stages is None:
            _check(load().vsie_profile(self._h, 1 if enable else 0))
        else:
            mask = 0
            for st in stages:
                mask |= 1 << STAGES.index(st)
            _check(load().vsie_profile_mask(self._h, C.c_uint32(mask if enable else 0)))

    def set_concurrency(self, enable=True):
        """Run the far-block chain of each product on a second stream (see vsie_set_concurrency)."""
        _check(load().vsie_set_concurrency(self._h, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total_ms, calls)} for stages that ran."""
        n = 16
        names = (C.c_char_p * n)()
        ms = (C.c_double * n)()
        calls = (C.c_int64 * n)()
        ns = C.c_int(0)
        _check(load().vsie_profile_read(self._h, n, names, ms, calls, C.byref(ns)))
        return {names[i].decode(): (ms[i], int(calls[i])) for i in range(ns.value) if calls[i] > 0}

    def port_current(self, port, x_host):
        x = np.ascontiguousarray(x_host, np.complex128)
        out = (C.c_double * 2)()
        _check(load().vsie_port_current(self._h, int(port), x.ctypes.data_as(C.POINTER(C.c_double)), out))
        return complex(out[0], out[1])

    def _export(self, kind, index=0):
        n = C.c_size_t(0)
        _check(load().vsie_export(self._h, kind, index, None, C.byref(n)))
        buf = (C.c_ubyte * n.value)()
        _check(load().vsie_export(self._h, kind, index, buf, C.byref(n)))
        return bytes(buf)

    def export_tt(self, chi):
        raw = self._export(X_TT_CORES, chi)
        r = np.frombuffer(raw[:12], np.int32)
        data = np.frombuffer(raw[12:], np.complex128)
        n1, n2, n3 = (int(v) for v in self.sizes.n)
        shapes = [(n1, r[0]), (r[0], n2, r[1]), (r[1], n3, r[2]), (r[2], self.m_far)]
        out, off = [], 0
        for s in shapes:
            k = int(np.prod(s))
            out.append(data[off:off + k].reshape(s).copy())
            off += k
        return out

    def export_aca(self):
        raw = self._export(X_ACA)
        k = int(np.frombuffer(raw[:4], np.int32)[0])
        data = np.frombuffer(raw[4:], np.complex128)
        U = data[:self.m_near * k].reshape(self.m_near, k).copy()
        V = data[self.m_near * k:].reshape(self.m_far, k).copy()
        return U, V

    def export_stencil(self):
        raw = self._export(X_STENCIL)
        base = np.frombuffer(raw[:12 * self.m_near], np.int32).reshape(self.m_near, 3).copy()
        W = np.frombuffer(raw[12 * self.m_near:], np.float64).reshape(self.m_near, 3, 5, 5, 5).copy()
        return base, W

    def export_ext_grid(self):
        raw = np.frombuffer(self._export(X_EXT_GRID), np.int32)
        return tuple(raw[:3]), tuple(raw[3:6]), tuple(raw[6:9])

    def export_generator(self):
        ne, _, _ = self.export_ext_grid()
        raw = np.frombuffer(self._export(X_GENERATOR), np.complex128)
        return raw.reshape(6, ne[2], ne[1], ne[0]).copy()

    def import_tt(self, chi, cores):
        G1, G2, G3, G4 = [np.ascontiguousarray(c, np.complex128) for c in cores]
        r = np.array([G1.shape[1], G2.shape[2], G3.shape[2]], np.int32)
        blob = r.tobytes() + G1.tobytes() + G2.tobytes() + G3.tobytes() + G4.tobytes()
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        _check(load().vsie_import(self._h, X_TT_CORES, int(chi), buf, len(blob)))
        s = Sizes()
        _check(load().vsie_sizes(self._h, C.byref(s)))
        self.sizes = s

    def import_aca(self, U, V):
        U = np.ascontiguousarray(U, np.complex128)
        V = np.ascontiguousarray(V, np.complex128)
        k = np.array([U.shape[1]], np.int32)
        blob = k.tobytes() + U.tobytes() + V.tobytes()
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        _check(load().vsie_import(self._h, X_ACA, 0, buf, len(blob)))

    def save_checkpoint(self, path):
        """Store the TT cores and ACA factors of the far coupling (eqs. (12), (14)) in a file keyed
        by the inputs that fix them."""
        _check(load().vsie_checkpoint_save(self._h, os.fsencode(path)))

    def load_checkpoint(self, path):
        """Replace the far-coupling factors by those of a checkpoint written for the same inputs."""
        _check(load().vsie_checkpoint_load(self._h, os.fsencode(path)))
        s = Sizes()
        _check(load().vsie_sizes(self._h, C.byref(s)))
        self.sizes = s


# layers of the learned preconditioner's network: (name, Cin, Cout, ReLU); parameters per layer are
# the weights [Cout][3][3][3][Cin] then the biases [Cout], in this order
NET_LAYERS = (("e1a", 8, 16, True), ("e1b", 16, 16, True), ("e2a", 16, 32, True), ("e2b", 32, 32, True),
              ("e3a", 32, 48, True), ("e3b", 48, 48, True), ("e4a", 48, 64, True), ("e4b", 64, 64, True),
              ("d3", 112, 48, True), ("d2", 80, 32, True), ("d1", 48, 16, True), ("out", 16, 6, False))


def _dev_ptr(t, dtype_name="float32"):
    import torch
    if t is None:
        return C.c_void_p(None)
    if not t.is_cuda or not t.is_contiguous() or t.dtype != getattr(torch, dtype_name):
        raise ValueError("contiguous %s device tensors only" % dtype_name)
    return C.c_void_p(t.data_ptr())


class ProductGraph:
    """vsie_graph_create: the products of several operators (each with its own fixed x and out
    tensors) captured into one HIP graph; launch() replays them all. Keep the operators and tensors
    alive while the graph is used."""

    def __init__(self, ops, xs, outs, stream=None):
        if not (len(ops) == len(xs) == len(outs)) or not ops:
            raise ValueError("one x and one out tensor per operator")
        dt = None
        for op, x, y in zip(ops, xs, outs):
            if x.dim() not in (1, 2) or x.shape[-1] != op.N or not x.is_contiguous() or not x.is_cuda:
                raise ValueError("x must be a contiguous device tensor [N] or [nrhs][N] of its operator")
            if y.shape != x.shape or y.dtype != x.dtype or not y.is_contiguous() or y.data_ptr() == x.data_ptr():
                raise ValueError("out must match x and not alias it")
            code = op._dtype_code(x)
            if dt is not None and code != dt:
                raise ValueError("all products in one precision")
            dt = code
        n = len(ops)
        hs = (C.c_void_p * n)(*[op._h.value for op in ops])
        nr = (C.c_int * n)(*[1 if x.dim() == 1 else x.shape[0] for x in xs])
        xp = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        yp = (C.c_void_p * n)(*[y.data_ptr() for y in outs])
        g = C.c_void_p()
        _check(load().vsie_graph_create(n, hs, dt, nr, xp, yp, _stream_ptr(stream), C.byref(g)))
        self._g = g
        self._keep = (ops, xs, outs)

    def launch(self, stream=None):
        _check(load().vsie_graph_launch(self._g, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_g", None):
            load().vsie_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The learned preconditioner's network (vsie_net_*): parameters, training pairs, training."""

    def __init__(self, seed=1, pair_capacity=0):
        h = C.c_void_p()
        _check(load().vsie_net_create(int(seed), int(pair_capacity), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().vsie_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(load().vsie_net_info(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(nparam=a.value, n_pairs=b.value, adam_steps=c.value)

    def get_params(self):
        n = self.info()["nparam"]
        out = np.zeros(n, np.float32)
        _check(load().vsie_net_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), n))
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, np.float32)
        _check(load().vsie_net_set_params(self._h, flat.ctypes.data_as(C.POINTER(C.c_float)), flat.size))

    @staticmethod
    def unflatten(flat):
        """{name.w: [Cout][3][3][3][Cin], name.b: [Cout]} views of a flat parameter vector."""
        out, off = {}, 0
        for name, ci, co, _ in NET_LAYERS:
            nw = co * 27 * ci
            out[name + ".w"] = flat[off:off + nw].reshape(co, 3, 3, 3, ci)
            off += nw
            out[name + ".b"] = flat[off:off + co]
            off += co
        return out

    @staticmethod
    def flatten(p):
        return np.concatenate([np.concatenate([np.asarray(p[n + ".w"]).ravel(), np.asarray(p[n + ".b"]).ravel()])
                               for n, _, _, _ in NET_LAYERS]).astype(np.float32)

    def collect(self, op, ports, restart=50, max_iter=1000, tol=1e-6, stream=None):
        pl = np.ascontiguousarray([int(p) for p in ports], np.int32)
        o = SolveOpts(tol, restart, max_iter, VSIE_SCHUR, 1e-3, 1, 0.1)
        n = C.c_int64()
        _check(load().vsie_net_collect(self._h, op._h, int(pl.size), pl.ctypes.data_as(C.POINTER(C.c_int32)),
                                       C.byref(o), C.byref(n), _stream_ptr(stream)))
        return n.value

    def train(self, epochs, lr=1e-3, seed=0, stream=None):
        loss = C.c_double()
        _check(load().vsie_net_train(self._h, int(epochs), float(lr), int(seed), C.byref(loss), _stream_ptr(stream)))
        return loss.value

    def attach(self, op):
        _check(load().vsie_net_attach(op._h, self._h))

    def forward(self, x, stream=None):
        """x: [D][H][W][8] float32 device tensor -> y [D][H][W][6]."""
        import torch
        D, H, W, _ = x.shape
        y = torch.empty((D, H, W, 6), dtype=torch.float32, device="cuda")
        _check(load().vsie_net_forward(self._h, D, H, W, _dev_ptr(x), _dev_ptr(y), _stream_ptr(stream)))
        return y

    def gradients(self, x, t, stream=None):
        D, H, W, _ = x.shape
        loss = C.c_double()
        g = np.zeros(self.info()["nparam"], np.float32)
        _check(load().vsie_net_gradients(self._h, D, H, W, _dev_ptr(x), _dev_ptr(t), C.byref(loss),
                                         g.ctypes.data_as(C.POINTER(C.c_float)), _stream_ptr(stream)))
        return loss.value, g

    def adam(self, lr, stream=None):
        _check(load().vsie_net_adam(self._h, float(lr), _stream_ptr(stream)))

    def layer(self, layer, mode, dims, in0, in1=None, mask=None, out=None, stream=None):
        D, H, W = dims
        _check(load().vsie_net_layer(self._h, int(layer), int(mode), D, H, W, _dev_ptr(in0), _dev_ptr(in1),
                                     _dev_ptr(mask), _dev_ptr(out), _stream_ptr(stream)))
        return out

    def layer_wgrad(self, layer, dims, in0, g, in1=None, mask=None, stream=None):
        D, H, W = dims
        _, ci, co, _ = NET_LAYERS[layer]
        gw = np.zeros((co, 27, ci), np.float32)
        gb = np.zeros(co, np.float32)
        _check(load().vsie_net_layer_wgrad(self._h, int(layer), D, H, W, _dev_ptr(in0), _dev_ptr(in1), _dev_ptr(g),
                                           _dev_ptr(mask), gw.ctypes.data_as(C.POINTER(C.c_float)),
                                           gb.ctypes.data_as(C.POINTER(C.c_float)), _stream_ptr(stream)))
        return gw.reshape(co, 3, 3, 3, ci), gb


LU_NOALLOC_MAX_N, LU_NOALLOC_MAX_NRHS = 4096, 64


def dense_lu_solve(A, B, stream=None, noalloc=False):
    """Solve A X = B on the device (complex128, row-major). A is overwritten by its LU factors and
    B by X; both are returned. noalloc selects vsie_dense_lu_solve_noalloc (static workspace,
    n <= LU_NOALLOC_MAX_N, nrhs <= LU_NOALLOC_MAX_NRHS)."""
    import torch
    if A.dtype != torch.complex128 or B.dtype != torch.complex128 or not (A.is_cuda and B.is_cuda):
        raise ValueError("complex128 device tensors only")
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
        raise ValueError("A must be square with unit column stride")
    Bm = B if B.dim() == 2 else B.view(-1, 1)
    if Bm.shape[0] != A.shape[0] or Bm.stride(1) != 1:
        raise ValueError("B must have n rows and unit column stride")
    fn = load().vsie_dense_lu_solve_noalloc if noalloc else load().vsie_dense_lu_solve
    _check(fn(A.shape[0], C.c_void_p(A.data_ptr()), A.stride(0), C.c_void_p(Bm.data_ptr()), Bm.stride(0), Bm.shape[1],
              _stream_ptr(stream)))
    return A, B
