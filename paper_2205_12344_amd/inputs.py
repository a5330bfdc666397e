"""Seeded synthetic inputs: media, forcing and problem presets.

This module holds no arithmetic of the method: it only draws materials and
sources, in float64 NumPy on the host, and is shared by the tests, the
benchmark and the CPU oracle's callers, so both sides see identical inputs.

The paper's workloads are analytic (Sec. 5: constant or piecewise media,
Gaussian and discrete-delta sources); nothing here stands in for a dataset.
Recipes (all seeded with numpy PCG64):

* Gaussian random field GRF(l, seed): white noise on a periodic grid padded
  by six correlation lengths, filtered in Fourier space by sqrt(S(k)) with
  S(k) ~ exp(-l^2 |k|^2 / 2) (Gaussian covariance, l = 0.1), cropped to the
  node grid and normalised to zero mean and unit sample standard deviation.
* Random log-normal media: rho = exp(0.2 g1), mu = exp(0.2 g2),
  lambda = mu * clip(2 exp(0.2 g3), 1, 3)  (median c_s ~ 1, c_p ~ 2).
* Three-layer 3-D medium along z: [0,1/3) c_s = 2, rho = 1.5; [1/3,2/3)
  c_s = 1.5, rho = 1.2; [2/3,1] c_s = 1, rho = 1; mu = rho c_s^2,
  lambda = 2 mu; each of rho, lambda, mu times (1 + 0.05 g), g a GRF clipped
  at +-3.
* Gaussian point sources  f(x) = exp(-|x - x0|^2 / (2 w^2)) e,  e a unit
  direction, amplitude 1 (the problem is linear).

Arrays use the node layout [component][z][y][x] (2-D: [c][y][x]) over
(n+1)^d nodes, x fastest.  Boundary faces are ordered -x,+x,-y,+y,-z,+z with
0 = Dirichlet, 1 = traction-free.
"""

import math
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

DIRICHLET = 0
FREE = 1
BC_ALL_DIRICHLET_2D = (0, 0, 0, 0)
BC_FREE_TOP_2D = (0, 0, 0, 1)        # Dirichlet sides and bottom, free top
BC_ABSORBING_Y_2D = (0, 0, 2, 2)     # Dirichlet sides, impedance bottom and top
BC_ABSORBING_2D = (2, 2, 2, 2)       # impedance on every face (an open box)
BC_ALL_DIRICHLET_3D = (0, 0, 0, 0, 0, 0)


@dataclass
class Case:
    name: str
    dim: int
    n: Tuple[int, ...]
    omega: float
    rho: np.ndarray
    lam: np.ndarray
    mu: np.ndarray
    f: np.ndarray
    bc: Tuple[int, ...]
    length: Tuple[float, ...] = None
    tol: float = 1e-10
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.length is None:
            self.length = (1.0,) * self.dim

    @property
    def h(self):
        return tuple(self.length[a] / self.n[a] for a in range(self.dim))

    @property
    def node_shape(self):
        return tuple(self.n[a] + 1 for a in reversed(range(self.dim)))


def _fast_len(m):
    """Smallest 2^a 3^b 5^c >= m (FFT friendly)."""
    best = None
    p2 = 1
    while p2 < 2 * m:
        p3 = p2
        while p3 < 2 * m:
            p5 = p3
            while p5 < 2 * m:
                if p5 >= m and (best is None or p5 < best):
                    best = p5
                p5 *= 5
            p3 *= 3
        p2 *= 2
    return best


def grf(node_shape, h, ell=0.1, seed=0, rng=None):
    """Gaussian random field on the node grid (see module docstring)."""
    import scipy.fft as sfft
    rng = np.random.default_rng(seed) if rng is None else rng
    dim = len(node_shape)
    hs = tuple(reversed(h)) if len(h) == dim else (h[0],) * dim   # per NumPy axis
    pad = [_fast_len(node_shape[k] + int(math.ceil(6 * ell / hs[k]))) for k in range(dim)]
    noise = rng.standard_normal(pad)
    spec = sfft.rfftn(noise, workers=-1)
    ks = []
    for k in range(dim):
        if k == dim - 1:
            kk = 2 * math.pi * np.fft.rfftfreq(pad[k], d=hs[k])
        else:
            kk = 2 * math.pi * np.fft.fftfreq(pad[k], d=hs[k])
        shape = [1] * dim
        shape[k] = kk.size
        ks.append(kk.reshape(shape))
    k2 = sum(kk * kk for kk in ks)
    spec *= np.exp(-0.25 * ell * ell * k2)           # sqrt of exp(-l^2 k^2 / 2)
    g = sfft.irfftn(spec, s=pad, workers=-1)
    g = g[tuple(slice(0, s) for s in node_shape)]
    g = g - g.mean()
    return g / g.std()


def media_random(node_shape, h, seed):
    """Random log-normal (rho, lambda, mu), correlation length 0.1, sigma 0.2,
    lambda / mu in [1, 3]."""
    rng = np.random.default_rng(seed)
    g1 = grf(node_shape, h, 0.1, rng=rng)
    g2 = grf(node_shape, h, 0.1, rng=rng)
    g3 = grf(node_shape, h, 0.1, rng=rng)
    rho = np.exp(0.2 * g1)
    mu = np.exp(0.2 * g2)
    lam = mu * np.clip(2.0 * np.exp(0.2 * g3), 1.0, 3.0)
    return rho, lam, mu


def media_layered3d(n, seed):
    """Three-layer medium along z with 5% smooth perturbations."""
    rng = np.random.default_rng(seed)
    shape = (n + 1,) * 3
    h = (1.0 / n,) * 3
    z = (np.arange(n + 1) / n).reshape(-1, 1, 1)
    cs = np.where(z < 1 / 3, 2.0, np.where(z < 2 / 3, 1.5, 1.0)) * np.ones(shape)
    rho0 = np.where(z < 1 / 3, 1.5, np.where(z < 2 / 3, 1.2, 1.0)) * np.ones(shape)
    mu0 = rho0 * cs * cs
    out = []
    for base in (rho0, 2.0 * mu0, mu0):
        g = np.clip(grf(shape, h, 0.1, rng=rng), -3.0, 3.0)
        out.append(base * (1.0 + 0.05 * g))
    rho, lam, mu = out
    return rho, lam, mu


def gaussian_sources(dim, n, length, centers, widths, directions):
    """Sum of Gaussian point sources, one direction vector per source."""
    shape = tuple(n[a] + 1 for a in reversed(range(dim)))
    coords = [np.arange(n[a] + 1) * (length[a] / n[a]) for a in range(dim)]
    grids = list(reversed(np.meshgrid(*[coords[a] for a in reversed(range(dim))], indexing="ij")))
    f = np.zeros((dim,) + shape)
    for x0, w, e in zip(centers, widths, directions):
        r2 = sum((grids[a] - x0[a]) ** 2 for a in range(dim))
        g = np.exp(-r2 / (2.0 * w * w))
        for c in range(dim):
            f[c] += e[c] * g
    return f


def unit_vector(rng, dim):
    v = rng.standard_normal(dim)
    return v / np.linalg.norm(v)


def min_shear_speed(rho, mu):
    return float(np.sqrt(np.asarray(mu) / np.asarray(rho)).min())


# --------------------------------------------------------------------------
# presets, shaped like the paper's experiments
# --------------------------------------------------------------------------

def constant_square64():
    """2-D unit square, 64 x 64 cells, rho = 1, lambda = 2, mu = 1, omega = 10,
    all Dirichlet; Gaussian of width 0.05 in x-displacement at (0.5, 0.5);
    CG to 1e-10."""
    n = (64, 64)
    shape = (65, 65)
    f = gaussian_sources(2, n, (1.0, 1.0), [(0.5, 0.5)], [0.05], [(1.0, 0.0)])
    return Case("square64_const", 2, n, 10.0, np.ones(shape), np.full(shape, 2.0),
                np.ones(shape), f, BC_ALL_DIRICHLET_2D, tol=1e-10)


def random_square(n=1024, seed=2, ppw=10.0):
    """2-D n x n cells, random log-normal media, omega for ~ppw points per
    shear wavelength at the slowest shear speed; Dirichlet sides and bottom,
    traction-free top; one seeded Gaussian of width 3.2 h."""
    h = 1.0 / n
    shape = (n + 1, n + 1)
    rho, lam, mu = media_random(shape, (h, h), seed)
    rng = np.random.default_rng(1000 + seed)
    x0 = rng.uniform(0.3, 0.7, size=2)
    e = unit_vector(rng, 2)
    f = gaussian_sources(2, (n, n), (1.0, 1.0), [x0], [3.2 * h], [e])
    omega = 2 * math.pi * min_shear_speed(rho, mu) / (ppw * h)
    return Case(f"square{n}_random", 2, (n, n), omega, rho, lam, mu, f, BC_FREE_TOP_2D,
                tol=1e-8, meta={"seed": seed, "center": x0.tolist(), "direction": e.tolist()})


def absorbing_square(n=1024, seed=2, ppw=10.0):
    """The random_square medium, source and omega with every face absorbing
    (impedance): an open box, the input of the two-field solve."""
    c = random_square(n, seed, ppw)
    c.name = f"square{n}_absorbing"
    c.bc = BC_ABSORBING_2D
    return c


def layered_cube(n=256, seed=3, ppw=8.0):
    """3-D n^3 cells, three-layer medium with 5% perturbations, all
    Dirichlet; omega for ~ppw points per shear wavelength; one Gaussian."""
    h = 1.0 / n
    rho, lam, mu = media_layered3d(n, seed)
    rng = np.random.default_rng(1000 + seed)
    x0 = rng.uniform(0.3, 0.7, size=3)
    e = unit_vector(rng, 3)
    f = gaussian_sources(3, (n, n, n), (1.0, 1.0, 1.0), [x0], [3.2 * h], [e])
    omega = 2 * math.pi * min_shear_speed(rho, mu) / (ppw * h)
    return Case(f"cube{n}_layered", 3, (n, n, n), omega, rho, lam, mu, f, BC_ALL_DIRICHLET_3D,
                tol=1e-8, meta={"seed": seed, "center": x0.tolist(), "direction": e.tolist()})


BC_FREE_Z_3D = (0, 0, 0, 0, 1, 1)    # Dirichlet sides, traction-free z = 0 and z = 1


def cube_bc_case(omega, free_z=False, h_omega=0.4, sigma_per_omega=10.0):
    """The boundary-condition experiment on the unit cube (Sec. 5.6): all
    Dirichlet, or traction-free z = 0 and z = 1 with Dirichlet elsewhere;
    h omega = 0.4 (n = round(omega / 0.4) cells per side), lambda = 2,
    mu = rho = 1, and per component j a Gaussian A_j exp(-sigma/2 |x - x_j|^2)
    with A_j = sigma^(3/2) and sigma = 10 omega (the section states only
    sigma ~ omega and A_j ~ sigma^(d/2)), the centres x_j slightly apart so
    that the forcing has both curl and divergence."""
    n = max(4, int(round(omega / h_omega)))
    shape = (n + 1,) * 3
    sigma = sigma_per_omega * omega
    centres = [(0.50, 0.50, 0.50), (0.53, 0.48, 0.51), (0.48, 0.52, 0.47)]
    c = np.arange(n + 1) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    f = np.zeros((3,) + shape)
    for j, (cx, cy, cz) in enumerate(centres):
        f[j] = sigma ** 1.5 * np.exp(-0.5 * sigma * ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2))
    one = np.ones(shape)
    bc = BC_FREE_Z_3D if free_z else BC_ALL_DIRICHLET_3D
    return Case(f"cube_bc_{'free' if free_z else 'dirichlet'}_w{omega:g}", 3, (n, n, n), omega, one, 2 * one, one,
                f, bc, tol=1e-9, meta={"sigma": sigma, "centres": centres})


def random_problem_2d(n, omega, seed, nsrc=None, width_h=(3.2, 3.2), rng=None):
    """One random 2-D problem: random log-normal media, 1-4 Gaussians in [0.2,0.8]^2."""
    h = 1.0 / n
    shape = (n + 1, n + 1)
    rho, lam, mu = media_random(shape, (h, h), seed)
    rng = np.random.default_rng(10_000 + seed) if rng is None else rng
    k = int(rng.integers(1, 5)) if nsrc is None else nsrc
    centers = [rng.uniform(0.2, 0.8, size=2) for _ in range(k)]
    dirs = [unit_vector(rng, 2) for _ in range(k)]
    widths = [rng.uniform(width_h[0], width_h[1]) * h for _ in range(k)]
    f = gaussian_sources(2, (n, n), (1.0, 1.0), centers, widths, dirs)
    return Case(f"rand2d_n{n}_s{seed}", 2, (n, n), float(omega), rho, lam, mu, f, BC_FREE_TOP_2D,
                tol=1e-8, meta={"seed": seed, "nsrc": k})


def ragged_batch(nprob=48, seed=4, nmin=256, nmax=1024, wmin=10.0, wmax=80.0):
    """Batch of problems with n ~ U{nmin..nmax}, omega ~ U[wmin, wmax]."""
    rng = np.random.default_rng(seed)
    cases = []
    for p in range(nprob):
        n = int(rng.integers(nmin, nmax + 1))
        om = float(rng.uniform(wmin, wmax))
        cases.append(random_problem_2d(n, om, seed=100 * seed + p))
    return cases


def warmstart_omega(seed):
    """The omega that warmstart_problem(seed) draws (its first draw)."""
    return float(np.random.default_rng(50_000 + seed).uniform(20.0, 60.0))


def warmstart_problem(seed, n=256):
    """Warm-start training/evaluation problem: n = 256, omega ~ U[20, 60],
    random log-normal media, 1-4 Gaussians of width U[2h, 6h]."""
    rng = np.random.default_rng(50_000 + seed)
    om = float(rng.uniform(20.0, 60.0))
    return random_problem_2d(n, om, seed=seed, width_h=(2.0, 6.0), rng=rng)


def random_field(shape, seed):
    """Plain standard-normal test vector (for operator-level parity tests)."""
    return np.random.default_rng(seed).standard_normal(shape)


# ---- mapped grids ------------------------------------------------------------

def sector_grid(nq, nr, n_an, arc=5.0):
    """Node coordinates (x, y), each of shape (nr + 1, nq + 1), of the annular
    sectors of the iterations-vs-frequency experiment (Sec. 5.5): q in [0, 1]
    runs radially from r_in to r_out = r_in + 1, r in [0, 1] along the arc,
    the outer arc has length `arc`; n_an = 1 is the quarter annulus
    (r_out = 2 arc / pi), n_an = 2 the half annulus (r_out = arc / pi)."""
    if n_an not in (1, 2):
        raise ValueError("n_an must be 1 (quarter) or 2 (half annulus)")
    r_out = 2.0 * arc / (n_an * math.pi)
    r_in = r_out - 1.0
    q = np.arange(nq + 1) / nq
    r = np.arange(nr + 1) / nr
    Q, R = np.meshgrid(q, r)
    rad = r_in + (r_out - r_in) * Q
    th = n_an * 0.5 * math.pi * R - 0.5 * math.pi
    return rad * np.cos(th), rad * np.sin(th)


def rectangle_grid(nq, nr, lq=1.0, lr=5.0):
    """Node coordinates of the lq x lr rectangle as a mapped grid (q along x)."""
    Q, R = np.meshgrid(np.arange(nq + 1) / nq, np.arange(nr + 1) / nr)
    return lq * Q, lr * R


def warped_grid(nq, nr, amp=0.06, seed=0):
    """A smooth, strongly non-orthogonal map of the unit square: the identity
    plus a seeded sum of low sine modes that vanish on no side (amplitude
    `amp`, small enough that the map stays one-to-one)."""
    rng = np.random.default_rng(seed)
    Q, R = np.meshgrid(np.arange(nq + 1) / nq, np.arange(nr + 1) / nr)
    x, y = Q.copy(), R.copy()
    for _ in range(3):
        kq, kr = rng.integers(1, 3, size=2)
        ph = rng.uniform(0, 2 * math.pi, size=2)
        c = rng.uniform(-1, 1, size=2)
        x += amp * c[0] * np.sin(math.pi * kq * Q + ph[0]) * np.cos(math.pi * kr * R + ph[1])
        y += amp * c[1] * np.cos(math.pi * kq * Q + ph[1]) * np.sin(math.pi * kr * R + ph[0])
    return x, y


def media_mapped(x, y, seed):
    """Random log-normal media (recipe above) on a mapped grid: the GRF is
    drawn on the (q, r) index grid with the correlation length measured in
    physical arc length along each direction's mean spacing."""
    shape = x.shape
    hq = float(np.mean(np.hypot(np.diff(x, axis=1), np.diff(y, axis=1))))
    hr = float(np.mean(np.hypot(np.diff(x, axis=0), np.diff(y, axis=0))))
    rng = np.random.default_rng(seed)
    gs = [grf(shape, (hq, hr), ell=0.1, rng=rng) for _ in range(3)]
    rho = np.exp(0.2 * gs[0])
    mu = np.exp(0.2 * gs[1])
    lam = mu * np.clip(2.0 * np.exp(0.2 * gs[2]), 1.0, 3.0)
    return rho, lam, mu


def sector_case(k, n_an=1, seed=None, arc=5.0):
    """The iterations-vs-frequency setup of Sec. 5.5 on an annular sector:
    omega = k + sqrt(2)/10, n_q = int(4 omega + 1) radial and
    n_r = int(4 arc omega + 1) arc-wise cells (about 20 points per shear
    wavelength), a discrete point source in u of amplitude omega^2 (divided
    by the cell's polar area) at node i = j = (n_q + 1) // 2.  Media:
    lambda = 2, mu = rho = 1 as in the paper, or (seed given) the random
    log-normal media above.  Returns (x, y, rho, lam, mu, omega, f)."""
    w = k + math.sqrt(2) / 10
    nq, nr = int(4 * w + 1), int(4 * arc * w + 1)
    x, y = sector_grid(nq, nr, n_an, arc)
    if seed is None:
        rho, lam, mu = np.ones(x.shape), 2.0 * np.ones(x.shape), np.ones(x.shape)
    else:
        rho, lam, mu = media_mapped(x, y, seed)
    r_out = 2.0 * arc / (n_an * math.pi)
    r_in = r_out - 1.0
    i = (nq + 1) // 2
    area = math.hypot(x[i, i], y[i, i]) * ((r_out - r_in) / nq) * (n_an * 0.5 * math.pi / nr)
    f = np.zeros((2,) + x.shape)
    f[0, i, i] = w * w / area
    return x, y, rho, lam, mu, w, f


def ring_grid(nq, nr, r_in=1.0, r_out=2.0, angle=math.pi):
    """Node coordinates of a ring sector with q along the arc and r radial
    (r = 0 the inner arc of radius r_in, r = 1 the outer arc of radius
    r_out; the angle decreases with q so the map is right-handed): the
    cross-section of the partial toroidal shell of Sec. 5.11 (1 <= r <= 2,
    0 <= theta <= pi), whose curved surfaces are traction-free."""
    Q, R = np.meshgrid(np.arange(nq + 1) / nq, np.arange(nr + 1) / nr)
    rad = r_in + (r_out - r_in) * R
    th = angle * (1.0 - Q)
    return rad * np.cos(th), rad * np.sin(th)


def torus_section(nq, nr, ns, R=4.0, r_in=1.0, r_out=2.0, theta=math.pi, phi=math.pi, phi0=0.0):
    """Node coordinates of a partial toroidal shell (the 3-D curvilinear
    experiment, Sec. 5.11):
        x = (R + r cos th) cos ph,  y = (R + r cos th) sin ph,  z = r sin th,
    with q -> ph in [phi0, phi0 + phi], r -> th in [0, theta], s -> r in
    [r_in, r_out] (the printed y uses cos ph, a typo: that map would fold).
    The orientation (q, r, s) = (ph, th, r) is right-handed.  Arrays of shape
    (ns + 1, nr + 1, nq + 1), q along the last axis."""
    q = np.linspace(0.0, 1.0, nq + 1)
    rr = np.linspace(0.0, 1.0, nr + 1)
    s = np.linspace(0.0, 1.0, ns + 1)
    S, Rr, Q = np.meshgrid(s, rr, q, indexing="ij")
    ph = phi0 + phi * Q
    th = theta * Rr
    rad = r_in + (r_out - r_in) * S
    x = (R + rad * np.cos(th)) * np.cos(ph)
    y = (R + rad * np.cos(th)) * np.sin(ph)
    z = rad * np.sin(th)
    return x, y, z
