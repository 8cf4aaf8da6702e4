"""Seeded synthetic workloads for the GMMNLSE propagation step.

This module only *generates inputs*: fibre constants, mode lists, the coupling
tensor of Eq. (2) for analytic Hermite-Gauss modes, Taylor dispersion
coefficients, sampled Raman response, launched pulses and step sizes.  It holds
none of the propagation arithmetic (no dispersion operator, no transforms, no
nonlinear operator, no integrator); both the HIP library and the CPU checker
receive what is built here as plain arrays.

Physical setting (Sec. III of the paper):
  * parabolic graded-index fibre (Sec. III.B "Graded-index"), whose modes form
    equally spaced groups (Sec. III.A, mode beating),
  * single linear polarisation with real scalar modes, so S^R = S^K is given by
    the overlap integral of Eq. (2),
  * dispersion as Taylor coefficients about omega_0 relative to the first mode
    (Eq. (1) and the paragraph after it).

The infinite parabolic profile n^2(r) = n_core^2 - NA^2 r^2 / a^2 has exact
Hermite-Gauss eigenmodes F = H_mx(sqrt2 x/w) H_my(sqrt2 y/w) exp(-r^2/w^2) with
w^2 = 2a/(k NA) and beta_g^2 = k^2 n_core^2 - 2 k (NA/a)(g+1), g = mx + my.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0          # m/s
N2_SILICA = 2.3e-20            # m^2/W, fused silica (assumed; the paper gives no value)
SEED_BASE = 170805324


def rng_for(cfg: int) -> np.random.Generator:
    """The seeded generator of workload ``cfg`` (draw order: phases, amplitudes, extras)."""
    return np.random.default_rng(SEED_BASE + int(cfg))


# ----------------------------------------------------------------------------- fibre + modes
@dataclass(frozen=True)
class GrinFiber:
    radius: float = 25e-6      # core radius a (m)
    na: float = 0.2            # numerical aperture
    lam0: float = 1030e-9      # centre wavelength (m)
    n_clad: float = 1.45

    @property
    def n_core(self) -> float:
        return math.sqrt(self.n_clad ** 2 + self.na ** 2)

    @property
    def omega0(self) -> float:
        return 2.0 * math.pi * C_LIGHT / self.lam0

    @property
    def k0(self) -> float:
        return 2.0 * math.pi / self.lam0

    @property
    def w(self) -> float:
        """1/e field radius of the fundamental Hermite-Gauss mode."""
        return math.sqrt(2.0 * self.radius / (self.k0 * self.na))


def hg_modes(n_groups: int) -> list[tuple[int, int]]:
    """Hermite-Gauss (mx, my) ordered by group g = mx + my, then mx descending."""
    out = []
    for g in range(n_groups):
        for mx in range(g, -1, -1):
            out.append((mx, g - mx))
    return out


def n_modes_for_groups(n_groups: int) -> int:
    return n_groups * (n_groups + 1) // 2


def _beta_group(fib: GrinFiber, g: int, omega: float) -> tuple[float, float]:
    """Propagation constant of group g and its first omega-derivative (exact)."""
    k = omega / C_LIGHT
    b2 = k * k * fib.n_core ** 2 - 2.0 * k * (fib.na / fib.radius) * (g + 1)
    b = math.sqrt(b2)
    db = (omega * fib.n_core ** 2 / C_LIGHT ** 2 - (fib.na / fib.radius) * (g + 1) / C_LIGHT) / b
    return b, db


def grin_betas(fib: GrinFiber, modes, beta2: float, n_beta: int = 3) -> np.ndarray:
    """Taylor coefficients [N][n_beta] in SI units (rad/m, s/m, s^2/m, ...).

    Column 0 is delta-beta_0, column 1 delta-beta_1, both relative to mode 0;
    column 2 is beta_2 (the same for every mode); higher columns are zero.
    """
    N = len(modes)
    out = np.zeros((N, n_beta))
    b_ref, db_ref = _beta_group(fib, modes[0][0] + modes[0][1], fib.omega0)
    for p, (mx, my) in enumerate(modes):
        b, db = _beta_group(fib, mx + my, fib.omega0)
        out[p, 0] = b - b_ref
        if n_beta > 1:
            out[p, 1] = db - db_ref
        if n_beta > 2:
            out[p, 2] = beta2
    return out


def _hermite_phys(n: int, x: np.ndarray) -> np.ndarray:
    """Physicists' Hermite polynomial H_n(x) by the three-term recurrence."""
    h0 = np.ones_like(x)
    if n == 0:
        return h0
    h1 = 2.0 * x
    for k in range(1, n):
        h0, h1 = h1, 2.0 * x * h1 - 2.0 * k * h0
    return h1


def coupling_tensor(fib: GrinFiber, modes, grid_n: int = 256, half_width: float = 40e-6) -> np.ndarray:
    """Eq. (2) on a grid_n x grid_n square grid of side 2*half_width, shape [N,N,N,N] (m^-2).

    The modes are products f_mx(x) f_my(y) and the grid is a tensor product, so
    the 2-D grid sums factor exactly into products of 1-D grid sums; they are
    evaluated that way (identical sums, fewer operations).
    """
    x = np.linspace(-half_width, half_width, grid_n)
    dx = x[1] - x[0]
    u = math.sqrt(2.0) * x / fib.w
    gmax = max(mx + my for mx, my in modes)
    f = np.stack([_hermite_phys(n, u) * np.exp(-(x / fib.w) ** 2) for n in range(gmax + 1)])
    f /= np.sqrt((f * f).sum(axis=1) * dx)[:, None]          # unit 1-D norm
    q = np.einsum("ax,bx,cx,dx->abcd", f, f, f, f) * dx       # 1-D quartic overlaps
    mx = np.array([m[0] for m in modes])
    my = np.array([m[1] for m in modes])
    S = (q[np.ix_(mx, mx, mx, mx)] * q[np.ix_(my, my, my, my)])
    return np.ascontiguousarray(S)


def raman_hR(nt: int, dt: float, tau1: float = 12.2e-15, tau2: float = 32e-15) -> np.ndarray:
    """Single damped-oscillator Raman response sampled at t = k*dt, k = 0..nt-1 (1/s)."""
    t = np.arange(nt) * dt
    return (tau1 ** 2 + tau2 ** 2) / (tau1 * tau2 ** 2) * np.exp(-t / tau2) * np.sin(t / tau1)


# ----------------------------------------------------------------------------- pulses
def time_grid(nt: int, dt: float) -> np.ndarray:
    """t_k = (k - nt/2) dt: the pulse is centred in the window."""
    return (np.arange(nt) - nt // 2) * dt


def sech_pulse(t, fwhm, peak_power):
    T0 = fwhm / (2.0 * math.acosh(math.sqrt(2.0)))
    return math.sqrt(peak_power) / np.cosh(t / T0) + 0j


def gaussian_pulse(t, fwhm, peak_power, chirp=0.0):
    T0 = fwhm / (2.0 * math.sqrt(math.log(2.0)))
    return math.sqrt(peak_power) * np.exp(-(1.0 + 1j * chirp) * t ** 2 / (2.0 * T0 ** 2))


def sech_peak_for_energy(fwhm, energy):
    T0 = fwhm / (2.0 * math.acosh(math.sqrt(2.0)))
    return energy / (2.0 * T0)


def gaussian_peak_for_energy(fwhm, energy):
    T0 = fwhm / (2.0 * math.sqrt(math.log(2.0)))
    return energy / (math.sqrt(math.pi) * T0)


# ----------------------------------------------------------------------------- workloads
@dataclass
class Workload:
    """Everything a propagation needs, as plain arrays and scalars (SI units)."""
    name: str
    nt: int
    dt: float
    omega0: float
    n2: float
    fR: float
    self_steepening: int
    betas: np.ndarray            # [N][n_beta]
    S: np.ndarray                # [N][N][N][N] real
    hR: np.ndarray | None        # [nt] or None when fR == 0
    A0: np.ndarray               # [N][nt] complex128, time domain, sqrt(W)
    dz: float
    L: float
    M: int
    extra: dict = field(default_factory=dict)

    @property
    def n_modes(self) -> int:
        return self.A0.shape[0]


def step_rule(gamma0000_peak: float, dbeta0_max: float) -> float:
    """Small step from the paper's length scales: min(z_NL/200, z_IM/5).

    z_NL = 1/(gamma P0) with all power in the fundamental (conservative) and
    z_IM = 1/max|delta beta_0| (step-size discussion of the parallel algorithm).
    """
    z_nl = 1.0 / gamma0000_peak
    z_im = 1.0 / dbeta0_max if dbeta0_max > 0 else float("inf")
    return min(z_nl / 200.0, z_im / 5.0)


def grin_workload(cfg: int, n_groups: int, nt: int, dt: float, pulse: str, fwhm: float,
                  energy: float | None = None, peak_power: float | None = None,
                  fractions=None, fR: float = 0.18, self_steepening: int = 1,
                  M: int = 10, L: float = 1.0, dz: float | None = None, beta2: float = 0.0187e-24,
                  random_complex: bool = False, chirp: float = 0.0, name: str = "",
                  fiber: GrinFiber | None = None) -> Workload:
    fib = fiber or GrinFiber()
    modes = hg_modes(n_groups)
    N = len(modes)
    betas = grin_betas(fib, modes, beta2)
    S = coupling_tensor(fib, modes)
    t = time_grid(nt, dt)
    rng = rng_for(cfg)
    if random_complex:
        c = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        c /= np.sqrt(np.sum(np.abs(c) ** 2))
    else:
        fr = np.full(N, 1.0 / N) if fractions is None else np.asarray(fractions, float)
        ph = rng.uniform(0.0, 2.0 * math.pi, N)
        c = np.sqrt(fr) * np.exp(1j * ph)
    if pulse == "sech":
        P0 = peak_power if peak_power is not None else sech_peak_for_energy(fwhm, energy)
        shape = sech_pulse(t, fwhm, 1.0)
    else:
        P0 = peak_power if peak_power is not None else gaussian_peak_for_energy(fwhm, energy)
        shape = gaussian_pulse(t, fwhm, 1.0, chirp)
    A0 = (math.sqrt(P0) * c[:, None] * shape[None, :]).astype(np.complex128)
    gamma0 = N2_SILICA * fib.omega0 / C_LIGHT * S[0, 0, 0, 0]
    if dz is None:
        dz = step_rule(gamma0 * P0, float(np.max(np.abs(betas[:, 0]))))
    hR = raman_hR(nt, dt) if fR > 0 else None
    return Workload(name=name or f"grin{cfg}", nt=nt, dt=dt, omega0=fib.omega0, n2=N2_SILICA, fR=fR,
                    self_steepening=self_steepening, betas=betas, S=S, hR=hR, A0=A0,
                    dz=dz, L=L, M=M, extra={"modes": modes, "P0": P0, "gamma0000": gamma0})


DT_FINE = 40e-12 / 2 ** 14      # 2.441 fs: the spacing used for Nt >= 2^12 windows


def config1() -> Workload:
    """3 modes (HG00, HG10, HG01), Kerr only, sech 100 fs / 10 kW, Nt=2^10 over 10 ps, dz=1 mm, L=0.5 m."""
    return grin_workload(1, 2, 2 ** 10, 10e-12 / 2 ** 10, "sech", 100e-15, peak_power=10e3,
                         fractions=[0.8, 0.1, 0.1], fR=0.0, self_steepening=0, M=10, L=0.5,
                         dz=1e-3, name="grin3_kerr_nt1024")


def config2(dz: float | None = None) -> Workload:
    """6 modes (groups 0-2), Kerr+Raman, 300 fs sech 50 nJ, Nt=2^13 over 20 ps, M=10, L=1 m."""
    return grin_workload(2, 3, 2 ** 13, 20e-12 / 2 ** 13, "sech", 300e-15, energy=50e-9, fR=0.18,
                         self_steepening=1, M=10, L=1.0, dz=dz, random_complex=True,
                         name="grin6_raman_nt8192")


def config3(dz: float | None = None) -> Workload:
    """15 modes (groups 0-4), Kerr+Raman, 200 fs Gaussian 100 nJ, Nt=2^14 over 40 ps, M=10, L=1 m."""
    return grin_workload(3, 5, 2 ** 14, DT_FINE, "gaussian", 200e-15, energy=100e-9, fR=0.18,
                         self_steepening=1, M=10, L=1.0, dz=dz, name="grin15_raman_nt16384")


def wide_workload(nt: int = 2 ** 15) -> Workload:
    """55 modes (groups 0-9), Kerr+Raman+shock, 200 fs Gaussian of 100 nJ over the
    modes, dt = 2.441 fs (Nt = 2^15: an 80 ps window), M = 10, dz by the rule:
    the largest request shape of the serving stream."""
    return grin_workload(9, 10, nt, DT_FINE, "gaussian", 200e-15, energy=100e-9, fR=0.18,
                         self_steepening=1, M=10, L=1.0, name=f"grin55_raman_nt{nt}")


def fig3_workload() -> Workload:
    """10 GRIN modes (groups 0-3), Nt = 2^14 over 40 ps, Kerr + Raman + shock, 200 fs
    Gaussian of 100 nJ over the modes, dz = z_NL / 200 (the ratio the timing
    comparison of the parallel algorithm quotes as typical)."""
    w = grin_workload(4, 4, 2 ** 14, DT_FINE, "gaussian", 200e-15, energy=100e-9, fR=0.18,
                      self_steepening=1, M=10, L=1.0, name="grin10_raman_nt16384")
    w.dz = 1.0 / (w.extra["gamma0000"] * w.extra["P0"]) / 200.0
    return w


def batch_problems(seed: int = 4, count: int = 64, length_scale: float = 1.0) -> list[Workload]:
    """The batched workload: `count` independent GRIN propagations, all drawn
    from numpy.random.default_rng(170805324 + seed) in this order per problem:
    Hermite-Gauss groups g in {2, 3, 4, 5} (3, 6, 10, 15 modes), log2 Nt in
    {12, 13, 14} (dt = 2.441 fs: windows of 10, 20, 40 ps), length uniform in
    [0.1, 1] m (times length_scale), energy log-uniform in [1, 200] nJ, linear
    chirp C uniform in [-5, 5] (a Gaussian of 200 fs FWHM with the phase
    exp(-i C t^2 / 2 T0^2), so its spectrum is sqrt(1 + C^2) times wider than
    transform-limited), then the mode phases.
    Equal energy over the modes, Kerr + Raman (fR = 0.18) + shock, M = 10, dz by
    the z_NL / z_IM rule."""
    rng = np.random.default_rng(SEED_BASE + seed)
    out = []
    for i in range(count):
        groups = int(rng.choice([2, 3, 4, 5]))
        logn = int(rng.choice([12, 13, 14]))
        L = float(rng.uniform(0.1, 1.0)) * length_scale
        E = float(np.exp(rng.uniform(np.log(1e-9), np.log(200e-9))))
        C = float(rng.uniform(-5.0, 5.0))
        fib = GrinFiber()
        modes = hg_modes(groups)
        N = len(modes)
        nt = 2 ** logn
        t = time_grid(nt, DT_FINE)
        ph = rng.uniform(0.0, 2.0 * math.pi, N)
        c = np.sqrt(np.full(N, 1.0 / N)) * np.exp(1j * ph)
        shape = gaussian_pulse(t, 200e-15, 1.0, C)
        P0 = E / (float(np.sum(np.abs(shape) ** 2)) * DT_FINE)   # peak power for energy E on the grid
        A0 = (math.sqrt(P0) * c[:, None] * shape[None, :]).astype(np.complex128)
        w = grin_workload(seed, groups, nt, DT_FINE, "gaussian", 200e-15, peak_power=P0, fR=0.18,
                          self_steepening=1, M=10, L=L, name=f"batch{i}_g{groups}_nt{nt}")
        w.A0 = A0
        w.extra.update({"energy": E, "chirp": C, "class": (N, nt)})
        out.append(w)
    return out


@dataclass
class Request:
    """One served propagation request."""
    idx: int
    arrival: float          # seconds after the start of the stream
    groups: int             # Hermite-Gauss groups (N = groups (groups + 1) / 2 modes)
    nt: int
    L: float
    A0: np.ndarray          # [N][nt] complex128 launch field
    energy: float
    chirp: float


def request_stream(seed: int = 5, count: int = 200, rate: float = 200.0, max_groups: int = 10,
                   length_scale: float = 0.01) -> list[Request]:
    """A seeded Poisson request stream of GRIN propagations: exponential gaps of
    mean 1/rate, then per request (draw order) Hermite-Gauss groups uniform in
    1..max_groups, log2 Nt uniform in 12..15 (dt = 2.441 fs), length uniform in
    [0.1, 2] m times length_scale, energy log-uniform in [1, 200] nJ, chirp
    uniform in [-5, 5] (200 fs FWHM Gaussian), mode phases; equal energy over
    the modes.  Kerr + Raman + shock and the step rule are the plan's and the
    server's (see serve.py)."""
    rng = np.random.default_rng(SEED_BASE + seed)
    gaps = rng.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        groups = int(rng.integers(1, max_groups + 1))
        nt = 2 ** int(rng.integers(12, 16))
        L = float(rng.uniform(0.1, 2.0)) * length_scale
        E = float(np.exp(rng.uniform(np.log(1e-9), np.log(200e-9))))
        C = float(rng.uniform(-5.0, 5.0))
        N = n_modes_for_groups(groups)
        ph = rng.uniform(0.0, 2.0 * math.pi, N)
        c = np.sqrt(np.full(N, 1.0 / N)) * np.exp(1j * ph)
        shape = gaussian_pulse(time_grid(nt, DT_FINE), 200e-15, 1.0, C)
        P0 = E / (float(np.sum(np.abs(shape) ** 2)) * DT_FINE)
        A0 = (math.sqrt(P0) * c[:, None] * shape[None, :]).astype(np.complex128)
        out.append(Request(i, float(arrivals[i]), groups, nt, L, A0, E, C))
    return out


def random_fields(seed: int, n_modes: int, nt: int, scale: float = 1.0) -> np.ndarray:
    """Smooth-ish random complex fields [N][nt] for operator-level parity checks."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    t = np.linspace(-1.0, 1.0, nt, endpoint=False)
    env = np.exp(-(t / 0.3) ** 2)
    a = (rng.standard_normal((n_modes, nt)) + 1j * rng.standard_normal((n_modes, nt))) * env
    return scale * a


def random_symmetric_tensor(seed: int, n_modes: int) -> np.ndarray:
    """A random real tensor with the full permutation symmetry of Eq. (2)."""
    rng = np.random.default_rng(SEED_BASE + 2000 + seed)
    X = rng.standard_normal((n_modes,) * 4)
    import itertools
    S = np.zeros_like(X)
    for perm in itertools.permutations(range(4)):
        S += np.transpose(X, perm)
    return S / 24.0


def random_general_tensor(seed: int, n_modes: int, complex_values: bool = True) -> np.ndarray:
    """A random tensor without any index symmetry (real or complex, entries of
    order one): the kind of S^K or S^R that polarised or complex modes give,
    for testing the general contraction route."""
    rng = np.random.default_rng(SEED_BASE + 3000 + seed)
    S = rng.standard_normal((n_modes,) * 4)
    if complex_values:
        S = S + 1j * rng.standard_normal((n_modes,) * 4)
    return S
