"""Python access to the reference oracle (plain serial FP64 C, ``oracle/*.c``).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use this module; the product path never
does.  It is a thin ctypes wrapper: every piece of arithmetic lives in the C
files, which follow arXiv 2211.14318 (Section 2 for W, P and the tangent
moduli, Algorithm 1 for the 1D hull, eq. 3.3 for lamination, eq. 5.2 /
Algorithm 3 for stresses and tangent moduli).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PLAIN = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
# R1_ORACLE_SANITIZE=1 loads the build under AddressSanitizer and UndefinedBehaviorSanitizer
# (build(sanitize=True)); the process must have the sanitizer runtime preloaded.
LIB = LIB_SAN if os.environ.get("R1_ORACLE_SANITIZE") == "1" else LIB_PLAIN
# sanitized build: the ROCm clang, so that one shared runtime serves it and the library's
# sanitized build in the same process
SAN_CC = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-fsanitize=address,undefined", "-shared-libsan", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]
SOURCES = ["energy.c", "hull.c", "lamination.c", "mlp.c", "grid.c", "path.c"]

MODEL_NH_DAMAGE = 0
MODEL_DOUBLEWELL = 1
MODEL_STVK_DAMAGE = 2
TREE_NODES = 3


def build(force=True, sanitize=False):
    """Compile the oracle with plain -O2 (no fast-math) against glibc libm; with
    sanitize=True, liboracle_san.so under AddressSanitizer and UndefinedBehaviorSanitizer."""
    out = LIB_SAN if sanitize else LIB_PLAIN
    if not force and os.path.exists(out):
        return out
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = [SAN_CC if sanitize else "gcc", "-O2", "-fno-fast-math", "-std=c99", "-Wall", "-Wextra", "-shared",
           "-fPIC", "-o", out + ".tmp"] + (SAN_FLAGS if sanitize else []) + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


class Material(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("model", ctypes.c_int), ("mu", ctypes.c_double),
                ("lam", ctypes.c_double), ("D_inf", ctypes.c_double), ("D0", ctypes.c_double)]


class Level(ctypes.Structure):
    _fields_ = [("n_dir", ctypes.c_int), ("a", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double)), ("n_t", ctypes.c_int),
                ("tau", ctypes.c_double)]


class Lamination(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("level", Level * 2)]


class Laminate(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_int), ("i_minus", ctypes.c_int), ("i_plus", ctypes.c_int),
                ("xi", ctypes.c_double), ("value", ctypes.c_double),
                ("dir_gap", ctypes.c_double), ("bridge_gap", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(sanitize=LIB == LIB_SAN)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_psi0.restype = ctypes.c_double
        L.orc_psi0.argtypes = [ctypes.POINTER(Material), dp]
        L.orc_damage.restype = ctypes.c_double
        L.orc_damage.argtypes = [ctypes.POINTER(Material), ctypes.c_double]
        L.orc_energy.restype = ctypes.c_double
        L.orc_energy.argtypes = [ctypes.POINTER(Material), dp, ctypes.c_double]
        L.orc_stress0.restype = ctypes.c_int
        L.orc_stress0.argtypes = [ctypes.POINTER(Material), dp, ctypes.c_double, dp]
        L.orc_tangent0.restype = ctypes.c_int
        L.orc_tangent0.argtypes = [ctypes.POINTER(Material), dp, ctypes.c_double, dp]
        L.orc_envelope_tangent.restype = ctypes.c_double
        L.orc_envelope_tangent.argtypes = [ctypes.POINTER(Material), ctypes.POINTER(Lamination), dp,
                                           ctypes.c_double, dp, dp, ctypes.POINTER(Laminate)]
        L.orc_eval_tree_tangent.restype = ctypes.c_double
        L.orc_eval_tree_tangent.argtypes = [ctypes.POINTER(Material), ctypes.POINTER(Lamination), dp,
                                            ctypes.c_double, ctypes.POINTER(Laminate), dp, dp]
        L.orc_envelope_batch_tangent.restype = None
        L.orc_envelope_batch_tangent.argtypes = [ctypes.POINTER(Material), ctypes.POINTER(Lamination),
                                                 ctypes.c_long, dp, dp, dp, dp, dp, ctypes.POINTER(Laminate)]
        L.orc_convexify.restype = ctypes.c_int
        L.orc_convexify.argtypes = [ctypes.c_int, dp, dp, ip]
        L.orc_hull_at_centre.restype = ctypes.c_double
        L.orc_hull_at_centre.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip, dp]
        L.orc_envelope.restype = ctypes.c_double
        L.orc_envelope.argtypes = [ctypes.POINTER(Material), ctypes.POINTER(Lamination), dp,
                                   ctypes.c_double, dp, ctypes.POINTER(Laminate)]
        L.orc_eval_tree.restype = ctypes.c_double
        L.orc_eval_tree.argtypes = [ctypes.POINTER(Material), ctypes.POINTER(Lamination), dp,
                                    ctypes.c_double, ctypes.POINTER(Laminate), dp]
        L.orc_envelope_batch.restype = None
        L.orc_envelope_batch.argtypes = [ctypes.POINTER(Material), ctypes.POINTER(Lamination),
                                         ctypes.c_long, dp, dp, dp, dp, ctypes.POINTER(Laminate)]
        L.orc_mlp_param_count.restype = ctypes.c_long
        L.orc_mlp_param_count.argtypes = [ctypes.c_int] * 4
        L.orc_mlp_forward.restype = ctypes.c_double
        L.orc_mlp_forward.argtypes = [ctypes.c_int] * 4 + [dp, ctypes.c_long, dp, dp, dp]
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        L.orc_mlp_loss_grad.argtypes = [ctypes.c_int] * 4 + [dp, ctypes.c_long, dp, dp, dp]
        gp = ctypes.POINTER(Grid)
        L.orc_grid_size.restype = ctypes.c_long
        L.orc_grid_size.argtypes = [gp]
        L.orc_grid_node.restype = None
        L.orc_grid_node.argtypes = [gp, ctypes.c_long, dp]
        L.orc_grid_r11.restype = ctypes.c_int
        L.orc_grid_r11.argtypes = [ctypes.c_int, ip]
        L.orc_grid_energy.restype = None
        L.orc_grid_energy.argtypes = [ctypes.POINTER(Material), gp, ctypes.c_double, dp, dp, dp]
        L.orc_grid_sweep.restype = ctypes.c_double
        L.orc_grid_sweep.argtypes = [gp, ctypes.c_int, ip, dp, dp, ctypes.c_int, dp, dp]
        L.orc_grid_update_node.restype = ctypes.c_double
        L.orc_grid_update_node.argtypes = [gp, ctypes.c_int, ip, dp, ctypes.c_long]
        L.orc_grid_laminate.restype = ctypes.c_int
        L.orc_grid_laminate.argtypes = [gp, ctypes.c_int, ip, dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, dp]
        L.orc_grid_interpolate.restype = ctypes.c_double
        L.orc_grid_interpolate.argtypes = [gp, dp, dp]
        L.orc_path_relax.restype = ctypes.c_int
        L.orc_path_relax.argtypes = [ctypes.POINTER(Material), ctypes.POINTER(Lamination), ctypes.c_int, dp,
                                     ctypes.c_double, ctypes.c_int, dp, dp, dp, ip]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def material(dim=2, model=MODEL_NH_DAMAGE, mu=1.0, lam=2.0, D_inf=0.99, D0=0.1):
    return Material(dim, model, mu, lam, D_inf, D0)


class LaminationSpec:
    """Keeps the direction arrays alive while the C struct points at them.

    levels: list of (a, b, n_t, tau), outermost first; a, b are (n_dir, dim)."""

    def __init__(self, levels):
        self._keep = []
        self.c = Lamination()
        self.c.depth = len(levels)
        for k, (a, b, n_t, tau) in enumerate(levels):
            a = np.ascontiguousarray(a, dtype=np.float64)
            b = np.ascontiguousarray(b, dtype=np.float64)
            assert a.shape == b.shape and n_t % 2 == 1
            self._keep += [a, b]
            self.c.level[k] = Level(a.shape[0], _dp(a), _dp(b), int(n_t), float(tau))
        self.levels = levels


def psi0(mat, G):
    G = np.ascontiguousarray(G, dtype=np.float64)
    return lib().orc_psi0(ctypes.byref(mat), _dp(G))


def damage(mat, beta):
    return lib().orc_damage(ctypes.byref(mat), float(beta))


def energy(mat, G, beta_n):
    G = np.ascontiguousarray(G, dtype=np.float64)
    return lib().orc_energy(ctypes.byref(mat), _dp(G), float(beta_n))


def stress0(mat, G, beta_n):
    G = np.ascontiguousarray(G, dtype=np.float64)
    P = np.empty_like(G)
    lib().orc_stress0(ctypes.byref(mat), _dp(G), float(beta_n), _dp(P))
    return P


def tangent0(mat, G, beta_n):
    """d^2 W / dG dG as a (d*d, d*d) array."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    dd = G.size
    A = np.empty((dd, dd))
    lib().orc_tangent0(ctypes.byref(mat), _dp(G), float(beta_n), _dp(A))
    return A


def envelope_tangent(mat, spec, F, beta_n, want_tree=False):
    """Returns (W^k, P^k (d x d), A^k (d*d x d*d), tree or None) for one point."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    dd = F.size
    P = np.empty_like(F)
    A = np.empty((dd, dd))
    tree = (Laminate * TREE_NODES)() if want_tree else None
    W = lib().orc_envelope_tangent(ctypes.byref(mat), ctypes.byref(spec.c), _dp(F), float(beta_n), _dp(P),
                                   _dp(A), tree)
    return W, P, A, (tree_to_list(tree) if want_tree else None)


def eval_tree_tangent(mat, spec, F, beta_n, nodes):
    """Energy, stress and tangent moduli of a given tree: nodes = list of (dir, i_minus, i_plus)."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    dd = F.size
    P = np.empty_like(F)
    A = np.empty((dd, dd))
    tree = (Laminate * TREE_NODES)()
    for k, (m, im, ip) in enumerate(nodes[:TREE_NODES]):
        tree[k].dir, tree[k].i_minus, tree[k].i_plus = int(m), int(im), int(ip)
    W = lib().orc_eval_tree_tangent(ctypes.byref(mat), ctypes.byref(spec.c), _dp(F), float(beta_n), tree,
                                    _dp(P), _dp(A))
    return W, P, A


def envelope_batch_tangent(mat, spec, F_soa, beta_n, want_tree=False):
    """SoA batch: F_soa (d*d, n), beta_n (n,) -> W (n,), P (d*d, n), A (d^4, n), trees."""
    F_soa = np.ascontiguousarray(F_soa, dtype=np.float64)
    beta_n = np.ascontiguousarray(beta_n, dtype=np.float64)
    dd, n = F_soa.shape
    W = np.empty(n)
    P = np.empty_like(F_soa)
    A = np.empty((dd * dd, n))
    trees = (Laminate * (TREE_NODES * n))() if want_tree else None
    lib().orc_envelope_batch_tangent(ctypes.byref(mat), ctypes.byref(spec.c), n, _dp(F_soa), _dp(beta_n),
                                     _dp(W), _dp(P), _dp(A), trees)
    if want_tree:
        t = tree_to_list(trees)
        trees = [t[p * TREE_NODES:(p + 1) * TREE_NODES] for p in range(n)]
    return W, P, A, trees


def convexify(x, w):
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    vert = np.empty(len(x), dtype=np.int32)
    n = lib().orc_convexify(len(x), _dp(x), _dp(w), vert.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return vert[:n].copy()


def hull_at_centre(w, c=None):
    w = np.ascontiguousarray(w, dtype=np.float64)
    if c is None:
        c = (len(w) - 1) // 2
    im, ip, gap = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    v = lib().orc_hull_at_centre(len(w), _dp(w), int(c), ctypes.byref(im), ctypes.byref(ip),
                                 ctypes.byref(gap))
    return v, im.value, ip.value, gap.value


def envelope(mat, spec, F, beta_n, want_tree=False):
    """Returns (W^k, P^k (d x d), tree or None) for one point."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    P = np.empty_like(F)
    tree = (Laminate * TREE_NODES)() if want_tree else None
    W = lib().orc_envelope(ctypes.byref(mat), ctypes.byref(spec.c), _dp(F), float(beta_n), _dp(P),
                           tree)
    return W, P, (tree_to_list(tree) if want_tree else None)


def tree_to_list(tree):
    return [dict(dir=t.dir, i_minus=t.i_minus, i_plus=t.i_plus, xi=t.xi, value=t.value,
                 dir_gap=t.dir_gap, bridge_gap=t.bridge_gap) for t in tree]


def eval_tree(mat, spec, F, beta_n, nodes):
    """Energy and stress of a given tree: nodes = list of (dir, i_minus, i_plus)."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    P = np.empty_like(F)
    tree = (Laminate * TREE_NODES)()
    for k, (m, im, ip) in enumerate(nodes[:TREE_NODES]):
        tree[k].dir, tree[k].i_minus, tree[k].i_plus = int(m), int(im), int(ip)
    W = lib().orc_eval_tree(ctypes.byref(mat), ctypes.byref(spec.c), _dp(F), float(beta_n), tree,
                            _dp(P))
    return W, P


def envelope_batch(mat, spec, F_soa, beta_n, want_stress=True, want_tree=False):
    """SoA batch: F_soa (d*d, n), beta_n (n,) -> W (n,), P (d*d, n), trees."""
    F_soa = np.ascontiguousarray(F_soa, dtype=np.float64)
    beta_n = np.ascontiguousarray(beta_n, dtype=np.float64)
    n = F_soa.shape[1]
    W = np.empty(n)
    P = np.empty_like(F_soa) if want_stress else None
    trees = (Laminate * (TREE_NODES * n))() if want_tree else None
    lib().orc_envelope_batch(ctypes.byref(mat), ctypes.byref(spec.c), n, _dp(F_soa), _dp(beta_n),
                             _dp(W), _dp(P) if want_stress else None, trees)
    if want_tree:
        t = tree_to_list(trees)
        trees = [t[p * TREE_NODES:(p + 1) * TREE_NODES] for p in range(n)]
    return W, P, trees


# ---- surrogate network oracle (mlp.c)

def mlp_param_count(d_in, width, n_hidden, d_out):
    return lib().orc_mlp_param_count(d_in, width, n_hidden, d_out)


def mlp_forward(shape, params, x, y=None):
    """shape = (d_in, width, n_hidden, d_out); x (B, d_in) -> (out (B, d_out), loss or None)."""
    d_in, width, n_hidden, d_out = shape
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty((x.shape[0], d_out))
    yy = np.ascontiguousarray(y, dtype=np.float64) if y is not None else None
    loss = lib().orc_mlp_forward(d_in, width, n_hidden, d_out, _dp(params), x.shape[0], _dp(x),
                                 _dp(yy) if yy is not None else None, _dp(out))
    return out, (loss if y is not None else None)


def mlp_loss_grad(shape, params, x, y):
    d_in, width, n_hidden, d_out = shape
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.empty_like(params)
    loss = lib().orc_mlp_loss_grad(d_in, width, n_hidden, d_out, _dp(params), x.shape[0], _dp(x),
                                   _dp(y), _dp(g))
    return loss, g


# ---- global lamination on a deformation-gradient mesh (grid.c)

class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 9), ("lo", ctypes.c_double * 9),
                ("delta", ctypes.c_double)]


def grid(dim, n, lo, delta):
    """Mesh with n[c] nodes lo[c] + k delta per component c = i*d + j."""
    g = Grid()
    g.dim = dim
    for c in range(dim * dim):
        g.n[c] = int(n[c])
        g.lo[c] = float(lo[c])
    g.delta = float(delta)
    return g


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def grid_size(g):
    return lib().orc_grid_size(ctypes.byref(g))


def grid_node(g, p):
    F = np.empty(g.dim * g.dim)
    lib().orc_grid_node(ctypes.byref(g), ctypes.c_long(p), _dp(F))
    return F.reshape(g.dim, g.dim)


def grid_r11(dim):
    steps = np.zeros((729, dim * dim), dtype=np.int32)
    k = lib().orc_grid_r11(dim, _ip(steps))
    return steps[:k].copy()


def grid_energy(mat, g, beta_n, stress=False, tangent=False):
    """W^0 at the nodes; with stress=True also P^0 (d*d, nodes), with tangent=True also
    the moduli (d^4, nodes)."""
    n, dd = grid_size(g), g.dim * g.dim
    W = np.empty(n)
    P = np.empty((dd, n)) if stress else None
    A = np.empty((dd * dd, n)) if tangent else None
    lib().orc_grid_energy(ctypes.byref(mat), ctypes.byref(g), float(beta_n), _dp(W), _dp(P) if stress else None,
                          _dp(A) if tangent else None)
    out = (W,) + ((P,) if stress else ()) + ((A,) if tangent else ())
    return out if len(out) > 1 else W


def grid_sweep(g, steps, Win, Pin=None):
    """One iteration; Pin (m, nodes): per-node quantities carried by the laminates."""
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    Win = np.ascontiguousarray(Win, dtype=np.float64)
    Wout = np.empty_like(Win)
    if Pin is None:
        md = lib().orc_grid_sweep(ctypes.byref(g), len(steps), _ip(steps), _dp(Win), _dp(Wout), 0, None, None)
        return Wout, md
    Pin = np.ascontiguousarray(Pin, dtype=np.float64)
    Pout = np.empty_like(Pin)
    md = lib().orc_grid_sweep(ctypes.byref(g), len(steps), _ip(steps), _dp(Win), _dp(Wout), Pin.shape[0],
                              _dp(Pin), _dp(Pout))
    return Wout, md, Pout


def grid_laminate(g, steps, W, k_max=20, tol=1e-4, P=None):
    """Returns (W, hist) or, with carried per-node quantities P (m, nodes), (W, hist, P)."""
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    W = np.array(W, dtype=np.float64)
    hist = np.zeros(max(k_max, 1))
    Pc = None if P is None else np.array(P, dtype=np.float64)
    k = lib().orc_grid_laminate(ctypes.byref(g), len(steps), _ip(steps), _dp(W), 0 if Pc is None else Pc.shape[0],
                                None if Pc is None else _dp(Pc), int(k_max), float(tol), _dp(hist))
    return (W, hist[:k].copy()) if Pc is None else (W, hist[:k].copy(), Pc)


def grid_interpolate(g, W, F):
    W = np.ascontiguousarray(W, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    return lib().orc_grid_interpolate(ctypes.byref(g), _dp(W), _dp(F))


def grid_update_node(g, steps, W, p):
    """Eq. 4.3 at node p alone (for sampled checks of large meshes)."""
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.float64)
    return lib().orc_grid_update_node(ctypes.byref(g), len(steps), _ip(steps), _dp(W), ctypes.c_long(p))


def path_relax(mat, spec, F_steps, beta0, fixed0=0):
    """Relax-then-fix driver of one point (path.c): F_steps (n_steps, d, d).  Returns
    W (n_steps,), P (n_steps, d, d), beta (n_steps,), fixed (n_steps,) and the step at
    which the envelope was fixed (-1 if never)."""
    F = np.ascontiguousarray(F_steps, dtype=np.float64)
    ns = F.shape[0]
    W = np.empty(ns)
    P = np.empty_like(F)
    beta = np.empty(ns)
    fixed = np.empty(ns, dtype=np.int32)
    first = lib().orc_path_relax(ctypes.byref(mat), ctypes.byref(spec.c), ns, _dp(F), float(beta0), int(fixed0),
                                 _dp(W), _dp(P), _dp(beta), fixed.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return W, P, beta, fixed, first
