"""Plain FP64 CPU oracle for the GMMNLSE and its massively parallel algorithm.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark import this module; the product (the HIP library
and its Python binding) never calls it and shares no code with it.

Everything is written out directly from the paper (Wright et al., "Multimode
Nonlinear Fiber Optics: Massively Parallel Numerical Solver, Tutorial and
Outlook"), in complex128, with numpy's FFT and matrix product as the only
library steps.  Three integrators of one operator:

  * ``mpa_propagate``  - the massively parallel algorithm (Sec. III.D: change of
    variables Eq. (cov), integral form Eq. (MPA_eq), M small steps inside one
    large step, trapezoid rule, fixed-point iteration to a threshold).
  * ``trapezoid_propagate`` - one small step at a time, the same trapezoid rule
    solved to round-off; the fixed point the converged MPA reaches for any M.
  * ``rk4ip_propagate`` - 4th-order Runge-Kutta in the interaction picture, an
    independent higher-order integrator of the same equation.

Conventions (readings of the paper; each is pinned by a test):
  * time grid t_k = (k - Nt/2) dt, angular frequency w_k = 2 pi fftfreq(Nt, dt);
  * a field is A(t) = sum_k A~(w_k) exp(-i w_k t), so d/dt <-> -i w.  This is the
    sign that makes D(t) of Sec. III.D become D_w = i(db0 + db1 w + sum b_m w^m/m!),
    makes (1 + (i/w0) d/dt) of Eq. (1) become (1 + w/w0) of Eq. (MPA_eq), and
    makes Eq. (8) a delay by +db1 z.  Spectrum = numpy ``ifft``, time = ``fft``;
  * the Raman convolution is circular on the window with weights
    h_R(k dt) dt renormalised to unit sum (zero-frequency gain exactly 1).
  * saturating gain (Sec. III.F, optional): the added terms are read as
    G_p = g_p [A_p - sum_lmn S^R_plmn A_l Phi_mn / I_sat],
    Phi_mn = int A_m A_n^* dtau.  The paper prints the saturation term without
    a gain factor; it comes from expanding g0 / (1 + F / F_sat) to first order
    and projecting on the modes, which leaves the gain coefficient in front of
    both terms (and makes the units those of g_p A_p, with I_sat a saturation
    fluence in J/m^2).  G enters the right-hand side beside the nonlinear term,
    without the factor i (n2 w0/c)(1 + (i/w0) d/dt).
  * linear mode coupling (Sec. III.F, optional): the added term
    C_p = i sum_n Q_np A_n with a z-independent coupling matrix Q, also beside
    the nonlinear term (so the MPA treats it inside its integrand, which needs
    L = M dz << 1/|Q|, the same regime as for the nonlinear length).
  * or, with ``Q_linear``, the same term moved into the linear operator: per
    frequency L(w) = diag(D_w) + i Q^T, an N x N matrix, and the change of
    variables of Sec. III.D uses its matrix exponential exp(L(w) z) in place of
    exp(D_w z).  C is linear and z-independent, so Eq. (cov) and Eq. (MPA_eq)
    carry over unchanged with that operator; the coupling is then exact for
    any step size and only the nonlinear term is left in the integrand.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

C_LIGHT = 299792458.0


# ----------------------------------------------------------------------------- model
@dataclass
class Model:
    """Inputs of Eq. (1) in SI units.

    betas : [N, nb] Taylor coefficients (db0, db1, b2, b3, ...) about omega0,
            db0/db1 relative to the first mode.
    SK, SR: [N, N, N, N] coupling tensors (Eq. (2) for real scalar modes;
            any real or complex tensor is accepted here).
    hR    : samples h_R(k dt), k = 0..Nt-1, or None when fR == 0.
    """
    betas: np.ndarray
    SK: np.ndarray
    SR: np.ndarray | None
    fR: float
    hR: np.ndarray | None
    dt: float
    omega0: float
    n2: float
    self_steepening: int = 1
    gain: np.ndarray | None = None   # [N] small-signal field gain g_p (1/m), or None
    I_sat: float = math.inf           # saturation fluence (J/m^2) of the gain term
    Q: np.ndarray | None = None      # [N, N] linear coupling Q_np (1/m), C_p = i sum_n Q_np A_n, or None
    Q_linear: bool = False           # True: C in the linear operator (matrix exponential), else in the integrand

    @property
    def n_modes(self) -> int:
        return self.betas.shape[0]

    @property
    def gamma_hat(self) -> float:
        """n2 omega0 / c, the prefactor of the nonlinear term in Eq. (1)."""
        return self.n2 * self.omega0 / C_LIGHT


def omega_grid(nt: int, dt: float) -> np.ndarray:
    return 2.0 * math.pi * np.fft.fftfreq(nt, dt)


def to_spectrum(A: np.ndarray) -> np.ndarray:
    """A~(w_k) = (1/Nt) sum_j A(t_j) exp(+i w_k t_j)  (numpy ifft)."""
    return np.fft.ifft(A, axis=-1)


def to_time(At: np.ndarray) -> np.ndarray:
    """A(t_j) = sum_k A~(w_k) exp(-i w_k t_j)  (numpy fft)."""
    return np.fft.fft(At, axis=-1)


def dispersion_operator(betas: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """D_w of Sec. III.D: F[D(t) A] = D_w A~ with d/dt -> -i w, shape [N, Nt].

    D(t) = i db0 - db1 d/dt + i sum_{n>=2} b_n/n! (i d/dt)^n   becomes
    D_w  = i (db0 + db1 w + sum_{n>=2} b_n w^n / n!).
    """
    nb = betas.shape[1]
    phase = np.zeros((betas.shape[0], omega.size))
    for n in range(nb):
        phase += betas[:, n:n + 1] * omega[None, :] ** n / math.factorial(n)
    return 1j * phase


def raman_transfer(hR: np.ndarray, dt: float) -> np.ndarray:
    """Spectral response of the causal Raman convolution of Eq. (1).

    R(t_j) = sum_k w_k B(t_{j-k}) with w_k = h_R(k dt) dt / sum_i h_R(i dt) dt,
    indices modulo Nt.  In spectrum space that is a multiplication by
    H = Nt * ifft(w) (so H[0] = 1).
    """
    w = hR * dt
    H = hR.size * np.fft.ifft(w)
    return H / H[0]


def raman_convolve_direct(hR: np.ndarray, B: np.ndarray) -> np.ndarray:
    """The same circular convolution as a plain double sum (small Nt only)."""
    nt = hR.size
    w = hR / hR.sum()
    out = np.zeros(B.shape, dtype=complex)
    for j in range(nt):
        for k in range(nt):
            out[..., j] += w[k] * B[..., (j - k) % nt]
    return out


def nonlinear_polarisation(A: np.ndarray, model: Model, H: np.ndarray | None) -> np.ndarray:
    """The bracket of Eq. (1), NL_p(t), for time-domain fields A [N, Nt].

    NL_p = sum_lmn (1-fR) SK_plmn A_l A_m A_n*  +  fR SR_plmn A_l (h_R * A_m A_n*)(t).
    The inner sums over (m, n) are one matrix product with S viewed as an
    (N^2 x N^2) matrix; the sum over l is then done explicitly.
    """
    N, nt = A.shape
    B = A[:, None, :] * np.conj(A[None, :, :])                  # B_mn(t) = A_m A_n^*
    SK = model.SK.reshape(N * N, N * N)
    CK = (SK @ B.reshape(N * N, nt)).reshape(N, N, nt)          # sum_mn SK_plmn B_mn
    NL = (1.0 - model.fR) * np.einsum("plt,lt->pt", CK, A)
    if model.fR != 0.0:
        R = to_time(H[None, None, :] * to_spectrum(B))           # h_R * B_mn
        SR = (model.SR if model.SR is not None else model.SK).reshape(N * N, N * N)
        CR = (SR @ R.reshape(N * N, nt)).reshape(N, N, nt)
        NL = NL + model.fR * np.einsum("plt,lt->pt", CR, A)
    return NL


def gain_term(A: np.ndarray, model: Model) -> np.ndarray:
    """Saturating gain of Sec. III.F for time-domain fields A [N, Nt]:
    G_p(t) = g_p [A_p(t) - sum_lmn S^R_plmn A_l(t) Phi_mn / I_sat],
    Phi_mn = int A_m A_n^* dtau (a rectangle-rule sum over the window)."""
    N = A.shape[0]
    g = np.asarray(model.gain, dtype=float)
    Phi = (A @ np.conj(A).T) * model.dt                           # Phi_mn = sum_t A_m A_n^* dt
    SR = model.SR if model.SR is not None else model.SK
    Msat = (SR.reshape(N * N, N * N) @ Phi.reshape(N * N)).reshape(N, N)   # sum_mn S^R_plmn Phi_mn
    return g[:, None] * (A - (Msat @ A) / model.I_sat)


def nonlinear_operator(At: np.ndarray, model: Model, omega: np.ndarray, H) -> np.ndarray:
    """N~[A](w) = i (n2 w0 / c) (1 + s w/w0) F{NL(t)}: the integrand factor of Eq. (MPA_eq),
    plus F{G} when the model has the saturating-gain term and F{C} with linear mode coupling."""
    A = to_time(At)
    NL = nonlinear_polarisation(A, model, H)
    shock = 1.0 + (omega / model.omega0 if model.self_steepening else 0.0)
    out = 1j * model.gamma_hat * shock * to_spectrum(NL)
    if model.gain is not None:
        out = out + to_spectrum(gain_term(A, model))
    if model.Q is not None and not model.Q_linear:
        out = out + 1j * (np.asarray(model.Q).T @ At)          # C_p = i sum_n Q_np A~_n (linear in A)
    return out


class _Ops:
    """Grid-dependent quantities of one model, built once per propagation."""

    def __init__(self, model: Model, nt: int):
        self.model = model
        self.omega = omega_grid(nt, model.dt)
        self.D = dispersion_operator(model.betas, self.omega)
        self.H = raman_transfer(model.hR, model.dt) if model.fR != 0.0 else None
        if model.self_steepening and np.any(1.0 + self.omega / model.omega0 <= 0.0):
            raise ValueError("window too fine: 1 + w/w0 <= 0 on the grid")

    def N(self, At):
        return nonlinear_operator(At, self.model, self.omega, self.H)

    def lin(self, z: float, At: np.ndarray) -> np.ndarray:
        """exp(L z) A~: the linear propagator over z (z may be negative).

        Diagonal case: exp(D_w z) A~.  With ``Q_linear``: per frequency the
        matrix exponential of L(w) z, L(w) = diag(D_w) + i Q^T, applied to the
        mode vector A~(w)."""
        if self.model.Q is None or not self.model.Q_linear:
            return np.exp(self.D * z) * At
        from scipy.linalg import expm
        key = float(z)
        cache = self.__dict__.setdefault("_expm", {})
        if key not in cache:
            Lw = np.zeros((self.omega.size,) + (self.D.shape[0],) * 2, dtype=np.complex128)
            Lw[:] = 1j * np.asarray(self.model.Q, dtype=np.complex128).T
            idx = np.arange(self.D.shape[0])
            Lw[:, idx, idx] += self.D.T
            cache[key] = expm(Lw * z)                   # [Nt, N, N]
        return np.einsum("kpq,qk->pk", cache[key], At)


def small_steps(L: float, dz: float) -> tuple[int, float]:
    """Number of small steps and the step actually used (L is covered exactly)."""
    r = L / dz
    n = int(round(r)) if abs(r - round(r)) < 1e-9 * max(1.0, r) else int(math.ceil(r))
    n = max(n, 1)
    return n, L / n


# ----------------------------------------------------------------------------- MPA
@dataclass
class MPAStats:
    large_steps: int = 0
    evaluations: int = 0
    iterations: list | None = None
    eps: list | None = None
    nonconverged: int = 0


def mpa_large_step(At0: np.ndarray, ops: _Ops, dz: float, M: int, tol: float = 1e-12,
                   max_iter: int = 20, fixed_iters: int = 0):
    """One large step L = M dz of the MPA from z0 (Sec. III.D).

    psi_p(z, w) = A~_p(z, w) exp[-D_w (z - z0)]   (Eq. (cov)) and, from Eq. (MPA_eq),
    psi(z_j) = psi(z0) + int_{z0}^{z_j} exp[-D_w (z'-z0)] N~[A(z')] dz'
    (with ``Q_linear``: exp(-L(w)(z - z0)) applied to the mode vector instead).
    Iterate: start from psi^(1)(z_j) = psi(z0); evaluate the integrands at all
    z_j (the parallel part); accumulate them with the trapezoid rule; repeat
    until the relative change of psi is below ``tol``.  Return A~(z0 + M dz).
    """
    psi0 = At0
    I0 = ops.N(At0)                                   # integrand at z0 (exp(-D*0) = 1)
    psi = [psi0.copy() for _ in range(M)]             # psi^(1)(z_j), j = 1..M
    n = 0
    eps_hist = []
    converged = False
    while True:
        n += 1
        I = [ops.lin(-j * dz, ops.N(ops.lin(j * dz, psi[j - 1]))) for j in range(1, M + 1)]
        new = []
        run = np.zeros_like(psi0)                     # sum_{k=1}^{j-1} I_k
        for j in range(1, M + 1):
            new.append(psi0 + dz * (0.5 * I0 + run + 0.5 * I[j - 1]))
            run = run + I[j - 1]
        diff = sum(np.sum(np.abs(a - b) ** 2) for a, b in zip(new, psi))
        size = sum(np.sum(np.abs(a) ** 2) for a in new)
        eps = math.sqrt(diff / size) if size > 0 else 0.0
        eps_hist.append(eps)
        psi = new
        if not math.isfinite(eps):                    # diverged: report, never loop on NaN
            break
        if fixed_iters:
            if n >= fixed_iters:
                converged = True
                break
        elif eps < tol:
            converged = True
            break
        elif n >= max_iter:
            break
    return ops.lin(M * dz, psi[M - 1]), n, eps_hist, converged


def mpa_propagate(A0: np.ndarray, model: Model, L: float, dz: float, M: int,
                  tol: float = 1e-12, max_iter: int = 20, fixed_iters: int = 0,
                  return_stats: bool = False):
    """Propagate time-domain fields A0 [N, Nt] over a fibre of length L.

    Large steps of M small steps; a final shorter large step takes the
    remaining n_small mod M small steps.  Returns the time-domain field at L.
    """
    ops = _Ops(model, A0.shape[1])
    n_small, dz = small_steps(L, dz)
    At = to_spectrum(A0.astype(np.complex128))
    st = MPAStats(iterations=[], eps=[])
    done = 0
    while done < n_small:
        m = min(M, n_small - done)
        At, n, eh, ok = mpa_large_step(At, ops, dz, m, tol, max_iter, fixed_iters)
        st.large_steps += 1
        st.evaluations += 1 + n * m
        st.iterations.append(n)
        st.eps.append(eh)
        st.nonconverged += 0 if ok else 1
        done += m
    out = to_time(At)
    return (out, st) if return_stats else out


# ----------------------------------------------------------------------------- serial trapezoid
def trapezoid_propagate(A0: np.ndarray, model: Model, L: float, dz: float,
                        tol: float = 1e-15, max_picard: int = 200):
    """Serial implicit trapezoid rule in the interaction picture, one dz at a time.

    Per step: psi1 = psi0 + dz/2 (N~[A0] + exp(-D dz) N~[exp(D dz) psi1]),
    solved by fixed-point iteration to round-off, then A~ <- exp(D dz) psi1.
    """
    ops = _Ops(model, A0.shape[1])
    n_small, dz = small_steps(L, dz)
    At = to_spectrum(A0.astype(np.complex128))
    for _ in range(n_small):
        f0 = ops.N(At)
        psi1 = At.copy()
        for _it in range(max_picard):
            nxt = At + 0.5 * dz * (f0 + ops.lin(-dz, ops.N(ops.lin(dz, psi1))))
            ch = np.linalg.norm(nxt - psi1) / max(np.linalg.norm(nxt), 1e-300)
            psi1 = nxt
            if ch < tol:
                break
        At = ops.lin(dz, psi1)
    return to_time(At)


# ----------------------------------------------------------------------------- RK4IP
def rk4ip_propagate(A0: np.ndarray, model: Model, L: float, dz: float):
    """4th-order Runge-Kutta in the interaction picture (Hult, JLT 25, 2007)."""
    ops = _Ops(model, A0.shape[1])
    n_small, h = small_steps(L, dz)
    Eh = lambda x: ops.lin(h / 2.0, x)                # noqa: E731  exp(L h/2)
    At = to_spectrum(A0.astype(np.complex128))
    for _ in range(n_small):
        AI = Eh(At)
        k1 = Eh(ops.N(At))
        k2 = ops.N(AI + 0.5 * h * k1)
        k3 = ops.N(AI + 0.5 * h * k2)
        k4 = ops.N(Eh(AI + h * k3))
        At = Eh(AI + h * (k1 / 6.0 + k2 / 3.0 + k3 / 3.0)) + h * k4 / 6.0
    return to_time(At)


# ----------------------------------------------------------------------------- invariants
def energy(A: np.ndarray, dt: float) -> float:
    """Total pulse energy sum_p int |A_p|^2 dt (J)."""
    return float(np.sum(np.abs(A) ** 2) * dt)


def photon_number(A: np.ndarray, dt: float, omega0: float) -> float:
    """Proportional to the photon number: sum_{p,k} |A~_p(w_k)|^2 / (w0 + w_k)."""
    At = to_spectrum(A)
    om = omega_grid(A.shape[-1], dt)
    return float(np.sum(np.abs(At) ** 2 / (omega0 + om)[None, :]))


def model_from_workload(w) -> Model:
    """Build a Model from a synthetic workload object (duck-typed)."""
    return Model(betas=np.asarray(w.betas, float), SK=np.asarray(w.S), SR=None, fR=float(w.fR),
                 hR=None if w.hR is None else np.asarray(w.hR, float), dt=float(w.dt),
                 omega0=float(w.omega0), n2=float(w.n2), self_steepening=int(w.self_steepening))
