"""Thin ctypes binding of libr1.so (C-ABI in include/r1.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Tensors are PyTorch device tensors (PyTorch is used
for device memory and streams); outputs are allocated here with torch and
filled by the library.  Importing this module fails loudly when the library
has not been built.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# R1_LIB_SANITIZE=1 loads the CPU-checking build (host C++ under AddressSanitizer and
# UndefinedBehaviorSanitizer, same kernels; python -m paper_2211_14318_amd.build --sanitize),
# which needs the sanitizer runtime preloaded into the process.
LIB_PATH = os.path.join(_PKG, "libr1_san.so" if os.environ.get("R1_LIB_SANITIZE") == "1" else "libr1.so")

R1_OK = 0
R1_F32, R1_F64 = 0, 1
R1_NEOHOOKE_DAMAGE, R1_TEST_DOUBLEWELL, R1_STVK_DAMAGE = 0, 1, 2
PT_DETLE0, PT_NONFINITE, PT_FALLBACK, PT_ITERCAP, PT_TIE = 1, 2, 4, 8, 16
TREE_NODES = 3


class R1Error(RuntimeError):
    def __init__(self, status, what, detail=""):
        super().__init__("%s failed: %s (%d)%s" % (what, _status_string(status), status,
                                                   (": " + detail) if detail else ""))
        self.status = status


class Material(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("model", ctypes.c_int32), ("mu", ctypes.c_double),
                ("lam", ctypes.c_double), ("D_inf", ctypes.c_double), ("D0", ctypes.c_double)]


class Level(ctypes.Structure):
    _fields_ = [("n_dir", ctypes.c_int32), ("a", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double)), ("n_t", ctypes.c_int32),
                ("tau", ctypes.c_double)]


class Lamination(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("level", Level * 2)]


class Laminate(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_int32), ("i_minus", ctypes.c_int32), ("i_plus", ctypes.c_int32),
                ("xi", ctypes.c_float)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("val_fraction", ctypes.c_float), ("energy_weight", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class TrainReport(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("train_loss", ctypes.c_float),
                ("val_loss", ctypes.c_float), ("ms", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 9), ("lo", ctypes.c_double * 9),
                ("delta", ctypes.c_double)]


def grid(dim, n, lo, delta):
    """Mesh description (r1_grid): n[c] nodes lo[c] + k*delta for component c = i*dim + j."""
    g = Grid()
    g.dim = dim
    for c in range(dim * dim):
        g.n[c] = int(n[c])
        g.lo[c] = float(lo[c])
    g.delta = float(delta)
    return g


def grid_size(g):
    s = 1
    for c in range(g.dim * g.dim):
        s *= g.n[c]
    return s


def grid_r11(dim):
    """Steps of the reduced direction set (eq. 5.1), (count, dim*dim) int32."""
    buf = (ctypes.c_int32 * (169 * 9))()
    cnt = ctypes.c_int32()
    s = _lib.r1_grid_r11(int(dim), buf, ctypes.byref(cnt))
    if s != 0:
        raise R1Error(s, "r1_grid_r11", "")
    return np.array(buf[:cnt.value * dim * dim], dtype=np.int32).reshape(cnt.value, dim * dim)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("%s is not built; run __graft_entry__.build() or "
                          "python -m paper_2211_14318_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.r1_create.argtypes = [ctypes.POINTER(vp), i32]
    L.r1_destroy.argtypes = [vp]
    L.r1_status_string.restype = ctypes.c_char_p
    L.r1_status_string.argtypes = [i32]
    L.r1_last_error.restype = ctypes.c_char_p
    L.r1_last_error.argtypes = [vp]
    L.r1_envelope.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i64, i32,
                              vp, vp, vp, vp, vp]
    L.r1_envelope_stress.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i64,
                                     i32, vp, vp, vp, vp, vp, vp, vp]
    L.r1_envelope_stress_noalloc.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i64,
                                             i32, vp, vp, vp, vp, vp, vp, vp]
    L.r1_path_step.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i64, i32, vp, vp, vp,
                               vp, vp, vp, vp, vp]
    L.r1_envelope_tangent.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i64,
                                      i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.r1_laminate_tangent.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i64,
                                      i32, vp, vp, vp, vp, vp, vp]
    L.r1_grid_r11.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.r1_grid_energy.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Grid), ctypes.c_double, i32, vp, vp,
                                 vp, vp]
    L.r1_grid_laminate.argtypes = [vp, ctypes.POINTER(Grid), i32, ctypes.POINTER(i32), i32, vp, vp, vp, i32,
                                   ctypes.c_double, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), vp]
    L.r1_grid_interpolate.argtypes = [vp, ctypes.POINTER(Grid), i32, vp, i64, vp, vp, vp]
    L.r1_envelope_batched.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i32,
                                      i64, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.r1_batched_plan_create.argtypes = [vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i32,
                                         i64, vp, i32, vp, ctypes.POINTER(vp)]
    L.r1_batched_plan_execute.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.r1_batched_plan_destroy.argtypes = [vp]
    L.r1_set_segment_width.argtypes = [vp, i32, i32]
    L.r1_tuning_export.argtypes = [vp, ctypes.c_void_p, i32, ctypes.POINTER(i32)]
    L.r1_tuning_import.argtypes = [vp, ctypes.c_void_p, i32]
    L.r1_get_segment_width.argtypes = [vp, i32, i32, i32, ctypes.POINTER(i32)]
    L.r1_autotune.argtypes = [vp, ctypes.POINTER(Material), i32, i32, vp, ctypes.POINTER(i32)]
    L.r1_autotune_inner.argtypes = [vp, ctypes.POINTER(Material), i32, i32, vp, ctypes.POINTER(i32)]
    L.r1_get_inner_segment_width.argtypes = [vp, i32, i32, i32, ctypes.POINTER(i32)]
    L.r1_timing_enable.argtypes = [vp, i32]
    L.r1_timing_reset.argtypes = [vp]
    L.r1_timing_query.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(i64)]
    fp = ctypes.POINTER(ctypes.c_float)
    L.r1_surrogate_create.argtypes = [vp, ctypes.POINTER(vp), i32, i32, i32, ctypes.c_uint64]
    L.r1_surrogate_destroy.argtypes = [vp]
    L.r1_surrogate_pack.argtypes = [vp, i32, i64, i32, vp, vp, vp, vp, vp, vp, vp]
    L.r1_surrogate_train.argtypes = [vp, vp, ctypes.POINTER(Material), vp, vp, i64,
                                     ctypes.POINTER(TrainCfg), ctypes.POINTER(TrainReport), vp]
    L.r1_surrogate_calibrate.argtypes = [vp, vp, ctypes.POINTER(Material), vp, vp, i64, ctypes.c_float,
                                         ctypes.c_float, ctypes.POINTER(i32), vp]
    L.r1_surrogate_predict.argtypes = [vp, vp, ctypes.POINTER(Material), vp, i64, vp, vp, vp, vp]
    L.r1_surrogate_set_check.argtypes = [vp, ctypes.c_float]
    L.r1_surrogate_check_offsets.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.r1_surrogate_infer.argtypes = [vp, vp, ctypes.POINTER(Material), ctypes.POINTER(Lamination), i64,
                                     i32, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp]
    L.r1_surrogate_param_count.argtypes = [vp, ctypes.POINTER(i64)]
    L.r1_surrogate_get_params.argtypes = [vp, fp, i64]
    L.r1_surrogate_set_params.argtypes = [vp, fp, i64]
    L.r1_surrogate_get_norm.argtypes = [vp, fp, fp, fp, fp]
    L.r1_surrogate_loss_grad.argtypes = [vp, vp, vp, vp, i64, vp, fp, vp]
    L.r1_surrogate_save.argtypes = [vp, ctypes.c_char_p]
    L.r1_surrogate_load.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_char_p]
    for name in ("r1_surrogate_create", "r1_surrogate_destroy", "r1_surrogate_pack", "r1_surrogate_train",
                 "r1_surrogate_calibrate", "r1_surrogate_infer", "r1_surrogate_predict", "r1_surrogate_set_check",
                 "r1_surrogate_check_offsets", "r1_surrogate_param_count",
                 "r1_surrogate_get_params", "r1_surrogate_set_params", "r1_surrogate_get_norm",
                 "r1_surrogate_loss_grad", "r1_surrogate_save", "r1_surrogate_load"):
        getattr(L, name).restype = i32
    for name in ("r1_autotune", "r1_autotune_inner", "r1_get_inner_segment_width", "r1_timing_enable", "r1_timing_reset", "r1_timing_query", "r1_create", "r1_destroy", "r1_envelope", "r1_envelope_stress",
                 "r1_envelope_tangent", "r1_laminate_tangent", "r1_envelope_batched", "r1_grid_r11",
                 "r1_envelope_stress_noalloc", "r1_path_step",
                 "r1_batched_plan_create", "r1_batched_plan_execute", "r1_batched_plan_destroy",
                 "r1_grid_energy", "r1_grid_laminate", "r1_grid_interpolate", "r1_set_segment_width", "r1_get_segment_width"):
        getattr(L, name).restype = i32
    return L


_lib = _load()


def lib():
    return _lib


def _status_string(s):
    return _lib.r1_status_string(int(s)).decode()


def material(dim=2, model=R1_NEOHOOKE_DAMAGE, mu=1.0, lam=2.0, D_inf=0.99, D0=0.1):
    return Material(dim, model, mu, lam, D_inf, D0)


def material_from(d, dim, model=R1_NEOHOOKE_DAMAGE):
    return Material(dim, model, d["mu"], d["lam"], d["D_inf"], d["D0"])


class LaminationSpec:
    """levels: list of dicts {a, b, n_t, tau} (outermost first); keeps arrays alive."""

    def __init__(self, levels):
        self._keep = []
        self.c = Lamination()
        self.c.depth = len(levels)
        for k, lv in enumerate(levels):
            a = np.ascontiguousarray(lv["a"], dtype=np.float64)
            b = np.ascontiguousarray(lv["b"], dtype=np.float64)
            self._keep += [a, b]
            self.c.level[k] = Level(a.shape[0], a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    int(lv["n_t"]), float(lv["tau"]))
        self.levels = levels
        self.depth = len(levels)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Handle:
    """One library handle bound to a device (not thread-safe)."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device
        h = ctypes.c_void_p()
        self._check(_lib.r1_create(ctypes.byref(h), int(device)), "r1_create", use_err=False)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.r1_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s, what, use_err=True):
        if s != R1_OK:
            detail = _lib.r1_last_error(self.h).decode() if use_err and getattr(self, "h", None) else ""
            raise R1Error(s, what, detail)

    def _stream(self, stream):
        if stream is None:
            stream = self.torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    def set_segment_width(self, n_t, lanes):
        self._check(_lib.r1_set_segment_width(self.h, int(n_t), int(lanes)), "r1_set_segment_width")

    def tuning(self):
        """The handle's tuned segment widths as an (k, 5) int32 array of records
        (n_t, dtype, dim, role, lanes), e.g. to keep them between runs."""
        cnt = ctypes.c_int32()
        self._check(_lib.r1_tuning_export(self.h, None, 0, ctypes.byref(cnt)), "r1_tuning_export")
        rec = np.zeros((cnt.value, 5), dtype=np.int32)
        if cnt.value:
            self._check(_lib.r1_tuning_export(self.h, rec.ctypes.data, cnt.value, ctypes.byref(cnt)),
                        "r1_tuning_export")
        return rec

    def set_tuning(self, records):
        """Installs records as returned by tuning() (all checked first)."""
        rec = np.ascontiguousarray(records, dtype=np.int32).reshape(-1, 5)
        self._check(_lib.r1_tuning_import(self.h, rec.ctypes.data if len(rec) else None, len(rec)),
                    "r1_tuning_import")

    def segment_width(self, n_t, dtype, dim):
        out = ctypes.c_int32()
        self._check(_lib.r1_get_segment_width(self.h, int(n_t), int(dtype), int(dim),
                                              ctypes.byref(out)), "r1_get_segment_width")
        return out.value

    def autotune(self, mat, n_t, dtype, stream=None):
        out = ctypes.c_int32()
        self._check(_lib.r1_autotune(self.h, ctypes.byref(mat), int(n_t), int(dtype),
                                     self._stream(stream), ctypes.byref(out)), "r1_autotune")
        return out.value

    def autotune_inner(self, mat, n_t, dtype, stream=None):
        out = ctypes.c_int32()
        self._check(_lib.r1_autotune_inner(self.h, ctypes.byref(mat), int(n_t), int(dtype),
                                           self._stream(stream), ctypes.byref(out)), "r1_autotune_inner")
        return out.value

    def inner_segment_width(self, n_t, dtype, dim):
        out = ctypes.c_int32()
        self._check(_lib.r1_get_inner_segment_width(self.h, int(n_t), int(dtype), int(dim),
                                                    ctypes.byref(out)), "r1_get_inner_segment_width")
        return out.value

    def timing(self, on=True):
        self._check(_lib.r1_timing_enable(self.h, int(bool(on))), "r1_timing_enable")

    def timing_reset(self):
        self._check(_lib.r1_timing_reset(self.h), "r1_timing_reset")

    def timing_query(self, kernel):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        self._check(_lib.r1_timing_query(self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
                    "r1_timing_query")
        return ms.value, cnt.value

    def _dtype_code(self, t):
        if t.dtype == self.torch.float32:
            return R1_F32
        if t.dtype == self.torch.float64:
            return R1_F64
        raise TypeError("F must be float32 or float64")

    def envelope(self, mat, spec, F, beta_n, stress=True, tree=False, flags=True, tangent=False,
                 stream=None):
        """F: (d*d, n) device tensor (SoA), beta_n: (n,).  Returns dict of device tensors;
        with tangent=True also A, the (d**4, n) tangent moduli dP_ij/dF_kl."""
        torch = self.torch
        n = F.shape[1]
        d = mat.dim
        assert F.shape[0] == d * d and F.is_contiguous() and beta_n.is_contiguous()
        assert beta_n.shape == (n,) and beta_n.dtype == F.dtype
        dt = self._dtype_code(F)
        dev = F.device
        W = torch.empty(n, dtype=F.dtype, device=dev)
        P = torch.empty((d * d, n), dtype=F.dtype, device=dev) if stress else None
        T = torch.empty((n, TREE_NODES, 4), dtype=torch.int32, device=dev) if tree else None
        fl = torch.empty(n, dtype=torch.int32, device=dev) if flags else None
        if tangent:
            A = torch.empty((d ** 4, n), dtype=F.dtype, device=dev)
            self._check(_lib.r1_envelope_tangent(self.h, ctypes.byref(mat), ctypes.byref(spec.c), n, dt,
                                                 _ptr(F), _ptr(beta_n), _ptr(W), _ptr(P), _ptr(A),
                                                 _ptr(T), _ptr(fl), self._stream(stream)),
                        "r1_envelope_tangent")
            return dict(W=W, P=P, A=A, tree=T, flags=fl)
        self._check(_lib.r1_envelope_stress(self.h, ctypes.byref(mat), ctypes.byref(spec.c), n, dt,
                                            _ptr(F), _ptr(beta_n), _ptr(W), _ptr(P), _ptr(T),
                                            _ptr(fl), self._stream(stream)),
                    "r1_envelope_stress")
        return dict(W=W, P=P, tree=T, flags=fl)

    def path_step(self, mat, spec, F, beta, fixed, W, P=None, tree=None, flags=None, stream=None):
        """One step of the relax-then-fix driver (r1_path_step): the relaxed potential
        at F with the history beta into W (and P, tree, flags); beta (n,) and fixed
        (n,) int32 are updated in place."""
        n = F.shape[1]
        assert F.is_contiguous() and beta.shape == (n,) and beta.dtype == F.dtype
        assert fixed.shape == (n,) and fixed.dtype == self.torch.int32 and W.shape == (n,)
        self._check(_lib.r1_path_step(self.h, ctypes.byref(mat), ctypes.byref(spec.c), n, self._dtype_code(F),
                                      _ptr(F), _ptr(beta), _ptr(fixed), _ptr(W), _ptr(P), _ptr(tree), _ptr(flags),
                                      self._stream(stream)), "r1_path_step")

    def laminate_tangent(self, mat, spec, F, beta_n, W, tree, stream=None):
        """Tangent moduli (d**4, n) of the given (n, 3, 4) int32 trees (Algorithm 3)."""
        n = F.shape[1]
        d = mat.dim
        assert F.shape[0] == d * d and F.is_contiguous() and beta_n.is_contiguous()
        assert W.shape == (n,) and W.dtype == F.dtype and tree.shape == (n, TREE_NODES, 4)
        assert tree.dtype == self.torch.int32 and tree.is_contiguous()
        A = self.torch.empty((d ** 4, n), dtype=F.dtype, device=F.device)
        self._check(_lib.r1_laminate_tangent(self.h, ctypes.byref(mat), ctypes.byref(spec.c), n,
                                             self._dtype_code(F), _ptr(F), _ptr(beta_n), _ptr(W),
                                             _ptr(tree), _ptr(A), self._stream(stream)),
                    "r1_laminate_tangent")
        return A

    def envelope_into(self, mat, spec, F, beta_n, W, P=None, tree=None, flags=None, stream=None):
        """Same, writing into caller-provided tensors (no allocation)."""
        dt = self._dtype_code(F)
        self._check(_lib.r1_envelope_stress(self.h, ctypes.byref(mat), ctypes.byref(spec.c),
                                            F.shape[1], dt, _ptr(F), _ptr(beta_n), _ptr(W),
                                            _ptr(P), _ptr(tree), _ptr(flags),
                                            self._stream(stream)),
                    "r1_envelope_stress")

    def envelope_noalloc_into(self, mat, spec, F, beta_n, W, P=None, tree=None, flags=None, stream=None):
        """r1_envelope_stress_noalloc into caller-provided tensors (the library
        allocates nothing; its fixed per-device workspace is used)."""
        self._check(_lib.r1_envelope_stress_noalloc(self.h, ctypes.byref(mat), ctypes.byref(spec.c),
                                                    F.shape[1], self._dtype_code(F), _ptr(F), _ptr(beta_n),
                                                    _ptr(W), _ptr(P), _ptr(tree), _ptr(flags),
                                                    self._stream(stream)),
                    "r1_envelope_stress_noalloc")

    def grid_energy(self, mat, g, beta_n, dtype, stress=False, tangent=False, stream=None):
        """W^0 at every node of mesh g: (nodes,) device tensor of torch dtype; with
        stress=True also P^0, (d*d, nodes); with tangent=True also the moduli,
        (d^4, nodes).  Returns W alone or the tuple (W[, P][, A])."""
        n, dd = grid_size(g), g.dim * g.dim
        W = self.torch.empty(n, dtype=dtype, device="cuda")
        P = self.torch.empty((dd, n), dtype=dtype, device="cuda") if stress else None
        A = self.torch.empty((dd * dd, n), dtype=dtype, device="cuda") if tangent else None
        dt = R1_F32 if dtype == self.torch.float32 else R1_F64
        self._check(_lib.r1_grid_energy(self.h, ctypes.byref(mat), ctypes.byref(g), float(beta_n), dt, _ptr(W),
                                        _ptr(P), _ptr(A), self._stream(stream)), "r1_grid_energy")
        out = (W,) + ((P,) if stress else ()) + ((A,) if tangent else ())
        return out if len(out) > 1 else W

    def grid_laminate(self, g, steps, W, k_max=20, tol=1e-4, P=None, A=None, stream=None):
        """Iterates eq. 4.3 in place on W (and the node stresses P and moduli A);
        returns the per-iteration maximal decreases."""
        steps = np.ascontiguousarray(steps, dtype=np.int32)
        n, dd = grid_size(g), g.dim * g.dim
        assert W.is_contiguous() and W.numel() == n
        assert P is None or (P.is_contiguous() and P.shape == (dd, n) and P.dtype == W.dtype)
        assert A is None or (A.is_contiguous() and A.shape == (dd * dd, n) and A.dtype == W.dtype)
        it = ctypes.c_int32()
        dec = (ctypes.c_double * int(k_max))()
        self._check(_lib.r1_grid_laminate(self.h, ctypes.byref(g), len(steps),
                                          steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          self._dtype_code(W), _ptr(W), _ptr(P), _ptr(A), int(k_max), float(tol),
                                          ctypes.byref(it), dec, self._stream(stream)), "r1_grid_laminate")
        return np.array(dec[:it.value])

    def grid_interpolate(self, g, W, F, stream=None):
        """Multilinear interpolation of node values W at points F (d*d, n)."""
        assert F.is_contiguous() and F.dtype == W.dtype
        n = F.shape[1]
        out = self.torch.empty(n, dtype=W.dtype, device=W.device)
        self._check(_lib.r1_grid_interpolate(self.h, ctypes.byref(g), self._dtype_code(W), _ptr(W), n, _ptr(F),
                                             _ptr(out), self._stream(stream)), "r1_grid_interpolate")
        return out

    def batched_plan(self, mat, table_specs, lam_idx, dtype, stream=None):
        return BatchedPlan(self, mat, table_specs, lam_idx, dtype, stream)

    def envelope_batched(self, mat, table_specs, lam_idx, F, beta_n, stress=False, tree=False,
                         flags=True, stream=None):
        torch = self.torch
        n = F.shape[1]
        d = mat.dim
        dt = self._dtype_code(F)
        arr = (Lamination * len(table_specs))(*[s.c for s in table_specs])
        dev = F.device
        W = torch.empty(n, dtype=F.dtype, device=dev)
        P = torch.empty((d * d, n), dtype=F.dtype, device=dev) if stress else None
        T = torch.empty((n, TREE_NODES, 4), dtype=torch.int32, device=dev) if tree else None
        fl = torch.empty(n, dtype=torch.int32, device=dev) if flags else None
        self._check(_lib.r1_envelope_batched(self.h, ctypes.byref(mat), arr, len(table_specs), n,
                                             _ptr(lam_idx), dt, _ptr(F), _ptr(beta_n), _ptr(W),
                                             _ptr(P), _ptr(T), _ptr(fl), self._stream(stream)),
                    "r1_envelope_batched")
        return dict(W=W, P=P, tree=T, flags=fl)


class BatchedPlan:
    """A plan of the uneven batch (r1_batched_plan_*): the table, the table indices
    (read once at creation) and the ordered work lists; execute() replays it."""

    def __init__(self, handle, mat, table_specs, lam_idx, dtype, stream=None):
        self.hd = handle
        self.mat = mat
        self.dim = mat.dim
        self.n = int(lam_idx.numel())
        self.dtype = dtype
        self._specs = list(table_specs)
        arr = (Lamination * len(self._specs))(*[s.c for s in self._specs])
        p = ctypes.c_void_p()
        code = R1_F32 if dtype == handle.torch.float32 else R1_F64
        handle._check(_lib.r1_batched_plan_create(handle.h, ctypes.byref(mat), arr, len(self._specs), self.n,
                                                  _ptr(lam_idx), code, handle._stream(stream), ctypes.byref(p)),
                      "r1_batched_plan_create")
        self.p = p

    def execute(self, F, beta_n, W, P=None, tree=None, flags=None, stream=None):
        """Writes into the given device tensors (graphs are kept per set of buffers)."""
        assert F.shape == (self.dim * self.dim, self.n) and F.dtype == self.dtype and F.is_contiguous()
        assert beta_n.shape == (self.n,) and W.shape == (self.n,)
        self.hd._check(_lib.r1_batched_plan_execute(self.p, _ptr(F), _ptr(beta_n), _ptr(W), _ptr(P), _ptr(tree),
                                                    _ptr(flags), self.hd._stream(stream)),
                       "r1_batched_plan_execute")

    def outputs(self, stress=False, tree=False, flags=True):
        torch = self.hd.torch
        d = self.dim
        return dict(W=torch.empty(self.n, dtype=self.dtype, device="cuda"),
                    P=torch.empty((d * d, self.n), dtype=self.dtype, device="cuda") if stress else None,
                    tree=torch.empty((self.n, TREE_NODES, 4), dtype=torch.int32, device="cuda") if tree else None,
                    flags=torch.empty(self.n, dtype=torch.int32, device="cuda") if flags else None)

    def close(self):
        if getattr(self, "p", None) and getattr(self.hd, "h", None):
            _lib.r1_batched_plan_destroy(self.p)
        self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_offsets(n_t):
    """Sample offsets of the surrogate's a-posteriori check for lines of n_t points."""
    buf = (ctypes.c_int32 * 32)()
    cnt = ctypes.c_int32()
    s = _lib.r1_surrogate_check_offsets(int(n_t), buf, ctypes.byref(cnt))
    if s != 0:
        raise R1Error(s, "r1_surrogate_check_offsets", "")
    return np.array(buf[:cnt.value], dtype=np.int64)


def tree_view(T):
    """(n, 3, 4) int32 tree tensor -> numpy arrays dir, i_minus, i_plus (int) and xi (float32)."""
    a = T.cpu().numpy()
    return a[..., 0], a[..., 1], a[..., 2], a[..., 3].view(np.float32)


class Surrogate:
    """Learned surrogate owned by a Handle (C-ABI r1_surrogate_*)."""

    def __init__(self, handle, dim=2, n_hidden=4, width=128, seed=0, _ptr=None):
        self.hd = handle
        self.dim = dim
        self.d_in = self.d_out = dim * dim + 1
        self.n_hidden, self.width = n_hidden, width
        if _ptr is None:
            p = ctypes.c_void_p()
            handle._check(_lib.r1_surrogate_create(handle.h, ctypes.byref(p), dim, n_hidden, width,
                                                   ctypes.c_uint64(seed)), "r1_surrogate_create")
            self.s = p
        else:
            self.s = _ptr

    def close(self):
        if getattr(self, "s", None):
            _lib.r1_surrogate_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, F, beta_n, W, P, stream=None):
        torch = self.hd.torch
        n = F.shape[1]
        X = torch.empty((n, self.d_in), dtype=torch.float32, device=F.device)
        Y = torch.empty((n, self.d_out), dtype=torch.float32, device=F.device)
        self.hd._check(_lib.r1_surrogate_pack(self.hd.h, self.dim, n, self.hd._dtype_code(F), _ptr(F),
                                              _ptr(beta_n), _ptr(W), _ptr(P), _ptr(X), _ptr(Y),
                                              self.hd._stream(stream)), "r1_surrogate_pack")
        return X, Y

    def train(self, mat, X, Y, epochs=10, batch=4096, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
              val_fraction=0.05, energy_weight=4.0, seed=0, stream=None):
        cfg = TrainCfg(epochs, batch, lr, betas[0], betas[1], eps, val_fraction, energy_weight, seed)
        rep = TrainReport()
        self.hd._check(_lib.r1_surrogate_train(self.hd.h, self.s, ctypes.byref(mat), _ptr(X), _ptr(Y),
                                               X.shape[0], ctypes.byref(cfg), ctypes.byref(rep),
                                               self.hd._stream(stream)), "r1_surrogate_train")
        return dict(steps=rep.steps, train_loss=rep.train_loss, val_loss=rep.val_loss, ms=rep.ms)

    def calibrate(self, mat, X, Y, tol=1e-3, quantile=0.99, stream=None):
        out = ctypes.c_int32()
        self.hd._check(_lib.r1_surrogate_calibrate(self.hd.h, self.s, ctypes.byref(mat), _ptr(X), _ptr(Y),
                                                   X.shape[0], tol, quantile, ctypes.byref(out),
                                                   self.hd._stream(stream)), "r1_surrogate_calibrate")
        return out.value

    def set_check(self, eps):
        """A-posteriori check of served values (r1_surrogate_set_check); 0 turns it off."""
        self.hd._check(_lib.r1_surrogate_set_check(self.s, ctypes.c_float(eps)), "r1_surrogate_set_check")

    def predict(self, mat, X, stream=None):
        """Raw network output on packed rows X (n, d_in): gate cell (-1 outside the
        training box), predicted W and predicted gap, device tensors."""
        torch = self.hd.torch
        n = X.shape[0]
        cell = torch.empty(n, dtype=torch.int32, device=X.device)
        w = torch.empty(n, dtype=torch.float32, device=X.device)
        g = torch.empty(n, dtype=torch.float32, device=X.device)
        self.hd._check(_lib.r1_surrogate_predict(self.hd.h, self.s, ctypes.byref(mat), _ptr(X), n, _ptr(cell),
                                                 _ptr(w), _ptr(g), self.hd._stream(stream)), "r1_surrogate_predict")
        return cell, w, g

    def infer(self, mat, fallback_spec, F, beta_n, stream=None, out=None):
        torch = self.hd.torch
        n = F.shape[1]
        d = self.dim
        if out is None:
            out = dict(W=torch.empty(n, dtype=F.dtype, device=F.device),
                       P=torch.empty((d * d, n), dtype=F.dtype, device=F.device),
                       flags=torch.empty(n, dtype=torch.int32, device=F.device))
        nfb = ctypes.c_int64()
        self.hd._check(_lib.r1_surrogate_infer(self.hd.h, self.s, ctypes.byref(mat),
                                               ctypes.byref(fallback_spec.c), n, self.hd._dtype_code(F),
                                               _ptr(F), _ptr(beta_n), _ptr(out["W"]), _ptr(out["P"]),
                                               _ptr(out["flags"]), ctypes.byref(nfb),
                                               self.hd._stream(stream)), "r1_surrogate_infer")
        out["n_fallback"] = nfb.value
        return out

    def param_count(self):
        c = ctypes.c_int64()
        _lib.r1_surrogate_param_count(self.s, ctypes.byref(c))
        return c.value

    def get_params(self):
        n = self.param_count()
        a = np.empty(n, dtype=np.float32)
        self.hd._check(_lib.r1_surrogate_get_params(self.s, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n),
                       "r1_surrogate_get_params")
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        self.hd._check(_lib.r1_surrogate_set_params(self.s, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                    a.size), "r1_surrogate_set_params")

    def norm(self):
        fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        xm, xs = np.empty(self.d_in, np.float32), np.empty(self.d_in, np.float32)
        ym, ys = np.empty(self.d_out, np.float32), np.empty(self.d_out, np.float32)
        _lib.r1_surrogate_get_norm(self.s, fp(xm), fp(xs), fp(ym), fp(ys))
        return dict(x_mean=xm, x_std=xs, y_mean=ym, y_std=ys)

    def loss_grad(self, Xn, Yn, stream=None):
        torch = self.hd.torch
        g = torch.empty(self.param_count(), dtype=torch.float32, device=Xn.device)
        loss = ctypes.c_float()
        self.hd._check(_lib.r1_surrogate_loss_grad(self.hd.h, self.s, _ptr(Xn), _ptr(Yn), Xn.shape[0], _ptr(g),
                                                   ctypes.byref(loss), self.hd._stream(stream)),
                       "r1_surrogate_loss_grad")
        return loss.value, g

    def save(self, path):
        self.hd._check(_lib.r1_surrogate_save(self.s, path.encode()), "r1_surrogate_save")

    @classmethod
    def load(cls, handle, path, dim=2, n_hidden=4, width=128):
        p = ctypes.c_void_p()
        handle._check(_lib.r1_surrogate_load(handle.h, ctypes.byref(p), path.encode()), "r1_surrogate_load")
        return cls(handle, dim, n_hidden, width, _ptr=p)
