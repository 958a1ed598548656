"""Seeded synthetic inputs for the rank-one lamination workloads.

This module only draws inputs: deformation gradients F, history values beta_n,
rank-one direction sets (a_m, b_m) and line grids (n_t, tau).  It holds none of
the method's arithmetic and imports neither the GPU library nor the oracle, so
both sides can be fed the same arrays.

Shapes follow the workloads of the study (see ``WORKLOADS``):
  F       float64 array (d*d, n), component-major SoA: F[i*d + j, p]
  beta_n  float64 array (n,)
  levels  list of dicts {a: (n_dir, d), b: (n_dir, d), n_t, tau}, outermost first
"""
import math

import numpy as np

SEED0 = 2211143180

MATERIAL = dict(mu=1.0, lam=2.0, D_inf=0.99, D0=0.1)


def rng_for(tag):
    return np.random.Generator(np.random.PCG64(SEED0 + int(tag)))


def angle_directions(n_a, n_b):
    """a = (cos ta, sin ta), b = (cos tb, sin tb) with ta = j*pi/n_a, tb = k*pi/n_b.

    Angles on [0, pi) so that no line is listed twice (a and -a give the same
    line on a symmetric t-grid).  4 x 4 gives the 16 directions of the reduced
    set of integer directions with entries in {-1, 0, 1} up to sign and
    normalisation; a-major ordering."""
    ta = np.arange(n_a) * math.pi / n_a
    tb = np.arange(n_b) * math.pi / n_b
    A = np.stack([np.cos(ta), np.sin(ta)], axis=1)
    B = np.stack([np.cos(tb), np.sin(tb)], axis=1)
    a = np.repeat(A, n_b, axis=0)
    b = np.tile(B, (n_a, 1))
    return a, b


def fibonacci_sphere(n):
    """Standard n-point Fibonacci sphere: z_i = 1-(2i+1)/n, phi_i = i*pi*(3-sqrt 5)."""
    i = np.arange(n)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(1.0 - z * z)
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def fibonacci_directions(n_a, n_b):
    A = fibonacci_sphere(n_a)
    B = fibonacci_sphere(n_b)
    return np.repeat(A, n_b, axis=0), np.tile(B, (n_a, 1))


def level(a, b, n_t, tau):
    assert n_t % 2 == 1 and n_t >= 3
    return dict(a=np.ascontiguousarray(a, np.float64), b=np.ascontiguousarray(b, np.float64),
                n_t=int(n_t), tau=float(tau))


def perturbed_identity(rng, n, d, sigma, det_min):
    """F = I + sigma*N(0,1) per entry, resampled until det F > det_min. Returns (d*d, n)."""
    out = np.empty((n, d, d))
    filled = 0
    while filled < n:
        m = max(2 * (n - filled), 16)
        G = np.eye(d)[None] + sigma * rng.standard_normal((m, d, d))
        ok = G[np.linalg.det(G) > det_min]
        k = min(len(ok), n - filled)
        out[filled:filled + k] = ok[:k]
        filled += k
    return np.ascontiguousarray(out.reshape(n, d * d).T)


def smooth_field(rng, x, n_modes=8):
    """Unit-variance random field on [0,1]^2: sum of n_modes random Fourier modes."""
    k = rng.normal(0.0, 2.0 * math.pi, size=(n_modes, 2))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    amp = math.sqrt(2.0 / n_modes)
    return amp * np.cos(x @ k.T + ph[None]).sum(axis=1)


def _cfg(name, dim, F, beta_n, levels, dtype, **extra):
    d = dict(name=name, dim=dim, material=dict(MATERIAL), F=F, beta_n=beta_n, levels=levels,
             dtype=dtype, n=F.shape[1])
    d.update(extra)
    return d


def config1(n=64):
    """2D plane strain FP64: F = I + 0.2 N (det > 0.2), beta_n = 0, 16 directions
    (4 x 4 angles), 201 points on [-1, 1], depth 1."""
    rng = rng_for(1)
    F = perturbed_identity(rng, n, 2, 0.2, 0.2)
    a, b = angle_directions(4, 4)
    return _cfg("plain-2d-fp64-n64-16x201-k1", 2, F, np.zeros(n), [level(a, b, 201, 1.0)],
                "f64")


def config2(n=4096, outer=(8, 8, 1025), inner=(8, 4, 257), tau=1.5, seed_tag=2):
    """2D: F = I + 0.3 N (det > 0.1), beta_n ~ U[0, 0.5]; outer 64 directions
    (8 x 8 angles) x 1025 points, inner 32 (8 x 4) x 257 points, tau = 1.5, depth 2."""
    rng = rng_for(seed_tag)
    F = perturbed_identity(rng, n, 2, 0.3, 0.1)
    beta_n = rng.uniform(0.0, 0.5, size=n)
    ao, bo = angle_directions(outer[0], outer[1])
    ai, bi = angle_directions(inner[0], inner[1])
    return _cfg("plain-2d-n%d-%dx%d-in%dx%d-k2" % (n, len(ao), outer[2], len(ai), inner[2]), 2, F,
                beta_n, [level(ao, bo, outer[2], tau), level(ai, bi, inner[2], tau)], "f32")


BATCH_NT = (257, 513, 1025, 2049)
BATCH_NDIR = ((8, 4), (8, 8), (16, 8))     # 32, 64, 128 directions
BATCH_DEPTH = (1, 2)


def config3_table(inner=(8, 4, 257), nts=BATCH_NT, ndirs=BATCH_NDIR, depths=BATCH_DEPTH):
    """Lamination table of the uneven batch: every (n_t, n_dir, depth) combination,
    tau = 1; depth-2 entries use an inner level of 32 directions x 257 points."""
    ai, bi = angle_directions(inner[0], inner[1])
    table = []
    for nt in nts:
        for (na, nb) in ndirs:
            a, b = angle_directions(na, nb)
            for k in depths:
                lv = [level(a, b, nt, 1.0)]
                if k == 2:
                    lv.append(level(ai, bi, inner[2], 1.0))
                table.append(lv)
    return table


def config3(n=65536, table=None):
    """65,536 2D points from three structured quad meshes of [0,1]^2 (64^2, 128^2,
    256^2 elements, one point per element), F as in config 1; beta_n is the
    small-strain energy proxy mu|E|^2 + lambda/2 (tr E)^2 of a prior-step strain
    field E = 0.2 S(x) made of smooth random fields S (a stand-in for a prior
    step's stored energy); uniform random (n_t, n_dir, depth) per point."""
    rng = rng_for(3)
    pts = []
    for ne in (64, 128, 256):
        h = 1.0 / ne
        g = (np.arange(ne) + 0.5) * h
        X, Y = np.meshgrid(g, g, indexing="ij")
        pts.append(np.stack([X.ravel(), Y.ravel()], axis=1))
    pts = np.concatenate(pts)
    sel = rng.choice(len(pts), size=n, replace=False)
    x = pts[sel]
    F = perturbed_identity(rng, n, 2, 0.2, 0.2)
    E = np.stack([0.2 * smooth_field(rng, x) for _ in range(4)], axis=0)  # (4, n)
    E12 = 0.5 * (E[1] + E[2])
    mu, lam = MATERIAL["mu"], MATERIAL["lam"]
    trE = E[0] + E[3]
    beta_n = np.maximum(0.0, mu * (E[0] ** 2 + E[3] ** 2 + 2 * E12 ** 2) + 0.5 * lam * trE ** 2)
    if table is None:
        table = config3_table()
    lam_idx = rng.integers(0, len(table), size=n).astype(np.int32)
    return _cfg("batched-2d-n%d" % n, 2, F, beta_n, None, "f32", table=table, lam_idx=lam_idx,
                coords=x)


def config4_training(n=2_000_000, seed_tag=40):
    """Surrogate training points: F = I + 0.4 N inside the training box
    (|F_ij - delta_ij| <= 1.2, det F > 0.1), beta_n ~ U[0, 1]; labels come from
    config-1-style lamination (16 x 201, tau = 1, depth 1)."""
    rng = rng_for(seed_tag)
    F = np.empty((4, 0))
    while F.shape[1] < n:
        G = perturbed_identity(rng, n, 2, 0.4, 0.1)
        keep = np.all(np.abs(G - np.array([1.0, 0, 0, 1.0])[:, None]) <= 1.2, axis=0)
        F = np.concatenate([F, G[:, keep]], axis=1)
    F = np.ascontiguousarray(F[:, :n])
    beta_n = rng.uniform(0.0, 1.0, size=n)
    a, b = angle_directions(4, 4)
    return _cfg("surrogate-train-2d-n%d" % n, 2, F, beta_n, [level(a, b, 201, 1.0)], "f32")


def config4_inference(n=1_000_000, seed_tag=41):
    """Inference points: F = I + 0.4 N (det > 0.1), beta_n ~ U[0, 1.1], so part of
    the batch lies outside the training box and falls back to lamination."""
    rng = rng_for(seed_tag)
    F = perturbed_identity(rng, n, 2, 0.4, 0.1)
    beta_n = rng.uniform(0.0, 1.1, size=n)
    a, b = angle_directions(4, 4)
    return _cfg("surrogate-infer-2d-n%d" % n, 2, F, beta_n, [level(a, b, 201, 1.0)], "f32")


def config5(n=262144, n_a=16, n_b=16, n_t=513, seed_tag=5):
    """3D FP32: F = I + 0.2 N (det > 0.2), beta_n ~ U[0, 0.5], 256 directions
    (16-point Fibonacci spheres for a and b), 513 points on [-1, 1], depth 1."""
    rng = rng_for(seed_tag)
    F = perturbed_identity(rng, n, 3, 0.2, 0.2)
    beta_n = rng.uniform(0.0, 0.5, size=n)
    a, b = fibonacci_directions(n_a, n_b)
    return _cfg("plain-3d-n%d-%dx%d-k1" % (n, len(a), n_t), 3, F, beta_n, [level(a, b, n_t, 1.0)],
                "f32")


def small_random(dim, n, n_dir_ab, n_t, tau=1.0, depth=1, inner=None, seed_tag=100, sigma=0.3,
                 det_min=0.1, beta_max=0.5):
    """Small parity cases with the structure of the workloads above."""
    rng = rng_for(seed_tag)
    F = perturbed_identity(rng, n, dim, sigma, det_min)
    beta_n = rng.uniform(0.0, beta_max, size=n)
    if dim == 2:
        a, b = angle_directions(*n_dir_ab)
    else:
        a, b = fibonacci_directions(*n_dir_ab)
    levels = [level(a, b, n_t, tau)]
    if depth == 2:
        na, nb, nt2 = inner
        ai, bi = angle_directions(na, nb) if dim == 2 else fibonacci_directions(na, nb)
        levels.append(level(ai, bi, nt2, tau))
    return _cfg("small-%dd-n%d" % (dim, n), dim, F, beta_n, levels, "f64")


PATH_AMPLITUDES = (0.0, 0.15, 0.3, 0.45, 0.6, 0.75, 0.9, 1.0, 0.85, 0.7, 0.55, 0.7, 0.9, 1.1, 1.3, 1.45)


BIAXIAL_MATERIAL = dict(mu=1.0, lam=0.5, D_inf=0.9, D0=0.3)    # neo-Hooke row of the biaxial test's table


def path_config(dim, n, n_dir_ab, n_t, tau=1.0, depth=1, inner=None, seed_tag=300, sigma=0.25,
                amplitudes=PATH_AMPLITUDES, beta_max=0.02, material=None):
    """Quadrature points driven along prescribed deformation paths (relax-then-fix
    driver): F_s = I + a_s H_p with one random H_p = sigma N(0,1) per point and a
    loading, unloading and reloading amplitude schedule a_s; H_p is redrawn until
    det F_s > 0.1 at every step.  beta_0 ~ U[0, beta_max].  F_steps has shape
    (n_steps, d*d, n), SoA per step.  Material: the biaxial test's neo-Hooke
    parameters unless given."""
    rng = rng_for(seed_tag)
    amp = np.asarray(amplitudes, dtype=np.float64)
    H = np.empty((n, dim, dim))
    filled = 0
    while filled < n:
        m = max(2 * (n - filled), 16)
        G = sigma * rng.standard_normal((m, dim, dim))
        ok = np.ones(m, dtype=bool)
        for a in amp:
            ok &= np.linalg.det(np.eye(dim)[None] + a * G) > 0.1
        G = G[ok]
        k = min(len(G), n - filled)
        H[filled:filled + k] = G[:k]
        filled += k
    F = np.eye(dim)[None, None] + amp[:, None, None, None] * H[None]      # (steps, n, d, d)
    F_steps = np.ascontiguousarray(F.reshape(len(amp), n, dim * dim).transpose(0, 2, 1))
    beta0 = rng.uniform(0.0, beta_max, size=n)
    if dim == 2:
        a, b = angle_directions(*n_dir_ab)
    else:
        a, b = fibonacci_directions(*n_dir_ab)
    levels = [level(a, b, n_t, tau)]
    if depth == 2:
        na, nb, nt2 = inner
        ai, bi = angle_directions(na, nb) if dim == 2 else fibonacci_directions(na, nb)
        levels.append(level(ai, bi, nt2, tau))
    d = dict(name="path-%dd-n%d-steps%d" % (dim, n, len(amp)), dim=dim,
             material=dict(BIAXIAL_MATERIAL if material is None else material),
             F_steps=F_steps, beta0=beta0, levels=levels, n=n, amplitudes=amp)
    return d
