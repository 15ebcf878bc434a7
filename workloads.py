"""Seeded synthetic workloads shaped like the paper's experiments.

This module only builds problem parameters and data arrays (closed-form
functions sampled on grids, seeded random draws).  It contains none of the
method's arithmetic and is shared by the CPU oracle tests, the GPU tests and
the benchmark.

Grid conventions (same as the library): sparse level L has finest level
J = L-1; the finest grid has nodes t_n = n T/2^J (n = 0..2^J) in time and the
2^J - 1 interior nodes x_m = m len/2^J per space axis; arrays are
[nt][ny][nx] (x fastest); data vanish on the spatial boundary.

Configurations (the paper publishes no data sets; every input is synthetic):
  c1  d=1, L=6,  c=1, T=1, u = sin(pi x) sin(pi t)  => f = 0, u0 = 0, v0 = pi sin(pi x)
  c2  d=1, L=12, T=2, c = 1 on (0,1/2), 1/2 on (1/2,1), f = 0,
      u0 = exp(-100 (x-0.3)^2), v0 = 0
  c3  d=2, L=10, c=1, T=1, u = sin(pi x) sin(pi y) sin(pi t)
      => f = pi^2 u, u0 = 0, v0 = pi sin(pi x) sin(pi y); adjoint seed g ~ N(0,1)
  c4  d=1, L=14, T=1, c on 8 cells ~ U[0.5,2]; a Gaussian source (width 0.05)
      for the observations plus N(0, 1e-3) noise; gradient at a second
      Gaussian with u0 = 0.1 sin(pi x), v0 = 0; 32 unit directions
  c5  256 problems d=2, L ~ U{6..10}, c on 4x4 blocks ~ U[0.5,2], f = sum of
      3 space-time Gaussians (width 0.05), u0 = v0 = 0, T = 1
"""

import math

import numpy as np


class Spec:
    """Problem parameters: d, lengths, ncell, c_vals (x fastest), T, L, and
    the coarsest level b0 of the combination (keyword; args() leaves it out)."""

    def __init__(self, d, lengths, ncell, c_vals, T, L, b0=1):
        self.d = int(d)
        self.lengths = [float(v) for v in lengths]
        self.ncell = [int(v) for v in ncell]
        self.c_vals = np.asarray(c_vals, dtype=np.float64).reshape(-1)
        self.T = float(T)
        self.L = int(L)
        self.b0 = int(b0)

    @property
    def J(self):
        return self.L - 1

    def nt(self):
        return 2 ** self.J + 1

    def nx(self):
        return 2 ** self.J - 1

    def shape(self):
        return (self.nt(),) + (self.nx(),) * self.d

    def space_shape(self):
        return (self.nx(),) * self.d

    def args(self):
        return (self.d, self.lengths, self.ncell, self.c_vals, self.T, self.L)

    def __repr__(self):
        return (f"Spec(d={self.d}, lengths={self.lengths}, ncell={self.ncell}, "
                f"T={self.T}, L={self.L}, b0={self.b0})")


def grids(spec):
    """(t, [x, y]) nodal coordinates of the finest grid."""
    J = spec.J
    t = spec.T * np.arange(2 ** J + 1) / 2 ** J
    xs = [spec.lengths[a] * np.arange(1, 2 ** J) / 2 ** J for a in range(spec.d)]
    return t, xs


def _space_mesh(spec):
    _, xs = grids(spec)
    if spec.d == 1:
        return (xs[0],)
    X = xs[0][None, :]
    Y = xs[1][:, None]
    return X, Y


def gaussian_source(spec, centres, width=0.05):
    """sum_m exp(-|(x,t) - z_m|^2 / (2 width^2)) sampled on the finest grid."""
    t, xs = grids(spec)
    out = np.zeros(spec.shape())
    for z in centres:
        gt = np.exp(-(t - z[-1]) ** 2 / (2 * width ** 2))
        gs = np.exp(-(xs[0] - z[0]) ** 2 / (2 * width ** 2))
        if spec.d == 2:
            gs = np.exp(-(xs[1][:, None] - z[1]) ** 2 / (2 * width ** 2)) * gs[None, :]
        out += gt.reshape((-1,) + (1,) * spec.d) * gs[None, ...]
    return out


# --------------------------------------------------------------- configs --

def c1():
    spec = Spec(1, [1.0], [1], [1.0], 1.0, 6)
    (x,) = _space_mesh(spec)
    f = np.zeros(spec.shape())
    return spec, dict(f=f, u0=np.zeros(spec.space_shape()), v0=math.pi * np.sin(math.pi * x))


def c2():
    spec = Spec(1, [1.0], [2], [1.0, 0.5], 2.0, 12)
    (x,) = _space_mesh(spec)
    return spec, dict(f=np.zeros(spec.shape()), u0=np.exp(-100.0 * (x - 0.3) ** 2),
                      v0=np.zeros(spec.space_shape()))


def c3(L=10, seed=0, with_cotangent=True):
    """d=2 manufactured problem; L may be lowered for small parity cases."""
    spec = Spec(2, [1.0, 1.0], [1, 1], [1.0], 1.0, L)
    t, _ = grids(spec)
    X, Y = _space_mesh(spec)
    s2 = np.sin(math.pi * X) * np.sin(math.pi * Y)
    f = (math.pi ** 2) * np.sin(math.pi * t)[:, None, None] * s2[None, :, :]
    data = dict(f=f, u0=np.zeros(spec.space_shape()), v0=math.pi * s2)
    if with_cotangent:
        data["g"] = np.random.default_rng(seed).standard_normal(spec.shape())
    return spec, data


def c4(L=14, seed=0):
    """Differentiation workload.  Draw order from default_rng(seed): 8 speeds,
    truth centre (x,t), gradient-point centre (x,t), noise array."""
    rng = np.random.default_rng(seed)
    cv = rng.uniform(0.5, 2.0, 8)
    spec = Spec(1, [1.0], [8], cv, 1.0, L)
    z_true = rng.uniform(0.0, 1.0, 2)
    z_eval = rng.uniform(0.0, 1.0, 2)
    noise = rng.normal(0.0, 1e-3, spec.shape())
    (x,) = _space_mesh(spec)
    return spec, dict(
        f_true=gaussian_source(spec, [z_true]),
        noise=noise,
        f=gaussian_source(spec, [z_eval]),
        u0=0.1 * np.sin(math.pi * x),
        v0=np.zeros(spec.space_shape()))


def c4_direction(spec, k, seed=0):
    """Direction k of the finite-difference check: N(0,1) entries over
    (f, u0) jointly, normalised to unit l2 norm (substream [seed, 1000+k])."""
    rng = np.random.default_rng([seed, 1000 + k])
    df = rng.standard_normal(spec.shape())
    du0 = rng.standard_normal(spec.space_shape())
    nrm = math.sqrt(float(np.sum(df * df) + np.sum(du0 * du0)))
    return df / nrm, du0 / nrm


def c5_specs(n=256, seed=0):
    """Parameters of the batch: per-problem L ~ U{6..10} and 4x4 speeds."""
    rng = np.random.default_rng(seed)
    Ls = rng.integers(6, 11, n)
    specs = []
    for i in range(n):
        cv = rng.uniform(0.5, 2.0, 16)
        specs.append(Spec(2, [1.0, 1.0], [4, 4], cv, 1.0, int(Ls[i])))
    return specs


def c5_centres(index, seed=0):
    """Centres (x, y, t) of problem `index`'s three Gaussians: the first draws
    of its substream [seed, index] (as in c5_data)."""
    return np.random.default_rng([seed, index]).uniform(0.0, 1.0, (3, 3))


def c5_data(spec, index, seed=0):
    """Data of problem `index`: f = sum of 3 Gaussians with centres from a
    per-problem substream; u0 = v0 = 0; cotangent g ~ N(0,1)."""
    rng = np.random.default_rng([seed, index])
    centres = rng.uniform(0.0, 1.0, (3, 3))
    f = gaussian_source(spec, centres)
    g = rng.standard_normal(spec.shape())
    z = np.zeros(spec.space_shape())
    return dict(f=f, u0=z, v0=z.copy(), g=g)


def random_data(spec, seed):
    """Generic seeded N(0,1) data (f, u0, v0, g) for parity cases."""
    rng = np.random.default_rng(seed)
    return dict(f=rng.standard_normal(spec.shape()),
                u0=rng.standard_normal(spec.space_shape()),
                v0=rng.standard_normal(spec.space_shape()),
                g=rng.standard_normal(spec.shape()))


# ------------------------------------------------- full-array parity sketches --
#
# A full-size array X is compared through k separable random projections
# s_k = <X, v_k0 (x) v_k1 (x) ...> with N(0,1) vectors per axis: for an error
# D, E[<D, v_0 (x) v_1 ...>^2] = ||D||^2, so the root mean square of the
# sketch differences estimates the whole-array l2 error without storing X,
# and an error anywhere (one slab, one tile) shows up.

def sketch_vectors(shape, k, seed=0):
    """Per-axis N(0,1) vectors of projection k (substream [seed, 7000 + k, axis])."""
    return [np.random.default_rng([seed, 7000 + k, ax]).standard_normal(n)
            for ax, n in enumerate(shape)]


def sketch(X, nproj=16, seed=0):
    """The nproj separable projections of X (any number of axes), contracting
    the last axis first."""
    X = np.asarray(X, dtype=np.float64)
    out = []
    for k in range(nproj):
        v = sketch_vectors(X.shape, k, seed)
        Y = X
        for ax in range(X.ndim - 1, -1, -1):
            Y = Y @ v[ax]
        out.append(float(Y))
    return out


def c4_cotangent(spec, seed=0):
    """A seeded N(0,1) cotangent of the differentiation workload's shape
    (substream [seed, 2000]): both sides run the adjoint on the same input."""
    return np.random.default_rng([seed, 2000]).standard_normal(spec.shape())
