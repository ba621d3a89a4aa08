"""Exact partition functions used to pin the oracle (test infrastructure only).

* ``brute_force``: enumerate all 2^N states of a small lattice (N <= 20) and
  return the density of states of the Hamiltonian of Eq. (4) with bond-wise
  couplings; written with numpy rolls, independently of the oracle's C code.
* ``kaufman_lnZ``: Kaufman's exact partition function of the L x L periodic
  Ising ferromagnet (Phys. Rev. 76, 1232 (1949); the four-term form as in
  Ferdinand & Fisher, Phys. Rev. 185, 832 (1969)), in mpmath.
* ``transfer_matrix_lnZ``: row-to-row transfer matrix for a 2D periodic lattice
  with arbitrary +-1 couplings, with per-row rescaling.
"""
import math

import mpmath as mp
import numpy as np


def site_grid(d, L):
    """Site index array shaped (L,)*d with the x coordinate on the last axis."""
    return np.arange(L ** d).reshape((L,) * d)


def neighbor_index(d, L, mu):
    """For each site s, the index of s + e_mu (periodic)."""
    g = site_grid(d, L)
    return np.roll(g, -1, axis=d - 1 - mu).reshape(-1)


def enumerate_states(d, L, J):
    """All 2^N spin states (N <= 20) as int8 rows, state c having sigma_s = -1
    where bit s of c is set, with their energies (Eq. (4), bond-wise J)."""
    N = L ** d
    if N > 20:
        raise ValueError("too many states")
    J = np.asarray(J, np.int64).reshape(N, d)
    c = np.arange(2 ** N, dtype=np.int64)[:, None]
    sigma = 1 - 2 * ((c >> np.arange(N)[None, :]) & 1)
    E = np.zeros(2 ** N, np.int64)
    for mu in range(d):
        nb = neighbor_index(d, L, mu)
        E -= (J[:, mu][None, :] * sigma * sigma[:, nb]).sum(axis=1)
    return sigma.astype(np.int8), E


def brute_force(d, L, J):
    """Density of states {E: count} over all 2^N spin states (N <= 20)."""
    _, E = enumerate_states(d, L, J)
    vals, cnt = np.unique(E, return_counts=True)
    return dict(zip(vals.tolist(), cnt.tolist()))


def lnZ_from_dos(dos, beta):
    """ln sum_E g(E) exp(-beta E), in mpmath."""
    return float(mp.log(mp.fsum(mp.mpf(g) * mp.exp(-mp.mpf(beta) * E) for E, g in dos.items())))


def mean_energy_from_dos(dos, beta):
    Z = mp.fsum(mp.mpf(g) * mp.exp(-mp.mpf(beta) * E) for E, g in dos.items())
    U = mp.fsum(mp.mpf(g) * E * mp.exp(-mp.mpf(beta) * E) for E, g in dos.items())
    return float(U / Z)


def kaufman_lnZ_mp(L, beta, J=1, dps=60):
    """ln Z of the L x L periodic Ising ferromagnet at coupling K = beta J (Kaufman 1949).

    Z = 1/2 (2 sinh 2K)^(N/2) [Z1 + Z2 + Z3 + Z4], N = L^2, with
      Z1 = prod_{r<L} 2 cosh(L g_{2r+1}/2),  Z2 = prod_{r<L} 2 sinh(L g_{2r+1}/2),
      Z3 = prod_{r<L} 2 cosh(L g_{2r}/2),    Z4 = prod_{r<L} 2 sinh(L g_{2r}/2),
    cosh g_l = cosh 2K coth 2K - cos(pi l / L) for l >= 1 and the signed
    g_0 = 2K + ln tanh K.  Returned as an mpmath number at ``dps`` digits.
    """
    with mp.workdps(dps):
        K = mp.mpf(beta) * mp.mpf(J)
        if K == 0:
            return L * L * mp.log(2)
        c = mp.cosh(2 * K) * mp.coth(2 * K)

        def g(l):
            if l == 0:
                return 2 * K + mp.log(mp.tanh(K))
            return mp.acosh(c - mp.cos(mp.pi * l / L))

        Z1 = mp.fprod(2 * mp.cosh(L * g(2 * r + 1) / 2) for r in range(L))
        Z2 = mp.fprod(2 * mp.sinh(L * g(2 * r + 1) / 2) for r in range(L))
        Z3 = mp.fprod(2 * mp.cosh(L * g(2 * r) / 2) for r in range(L))
        Z4 = mp.fprod(2 * mp.sinh(L * g(2 * r) / 2) for r in range(L))
        return mp.log(mp.mpf(1) / 2 * (2 * mp.sinh(2 * K)) ** (mp.mpf(L * L) / 2) *
                      (Z1 + Z2 + Z3 + Z4))


def kaufman_lnZ(L, beta, J=1):
    """Kaufman's ln Z as a double."""
    return float(kaufman_lnZ_mp(L, beta, J))


def kaufman_energy(L, beta, h=mp.mpf("1e-12")):
    """<E> = -d ln Z / d beta, central difference of the 60-digit ln Z."""
    with mp.workdps(60):
        b = mp.mpf(beta)
        return float(-(kaufman_lnZ_mp(L, b + h) - kaufman_lnZ_mp(L, b - h)) / (2 * h))


def transfer_matrix_lnZ(L, J, beta):
    """ln Z of a 2D L x L periodic lattice with couplings J[s*2+mu] (s = x + L y).

    Row states a in {0..2^L-1} (bit x set -> sigma = -1).  T_y[a, b] =
    exp(beta H_y(a)) exp(beta V_y(a, b)) with H_y the in-row bonds of row y and
    V_y the bonds between rows y and y+1; Z = Tr prod_y T_y.
    """
    J = np.asarray(J, np.float64).reshape(L * L, 2)
    a = np.arange(2 ** L)[:, None]
    sig = (1 - 2 * ((a >> np.arange(L)[None, :]) & 1)).astype(np.float64)  # (2^L, L)
    P = None
    logscale = 0.0
    for y in range(L):
        Jh = J[y * L + np.arange(L), 0]
        Jv = J[y * L + np.arange(L), 1]
        H = (Jh[None, :] * sig * np.roll(sig, -1, axis=1)).sum(axis=1)  # (2^L,)
        V = (sig * Jv[None, :]) @ sig.T  # (2^L, 2^L): sum_x Jv sigma_a,x sigma_b,x
        T = np.exp(beta * (H[:, None] + V) - beta * 2 * L)
        logscale += beta * 2 * L
        P = T if P is None else P @ T
        m = P.max()
        P = P / m
        logscale += math.log(m)
    return logscale + math.log(np.trace(P))


def beta_c():
    """Critical coupling of the 2D square-lattice Ising model, (1/2) ln(1 + sqrt 2)."""
    return 0.5 * math.log(1.0 + math.sqrt(2.0))


def kaufman_e_c(L, beta):
    """Energy and specific heat per spin, e = <E>/N and c = beta^2 Var(E)/N, from
    central differences (step 1e-15) of the 60-digit Kaufman ln Z."""
    N = L * L
    with mp.workdps(60):
        b, h = mp.mpf(beta), mp.mpf("1e-15")
        l0, lp, lm = (kaufman_lnZ_mp(L, x) for x in (b, b + h, b - h))
        return float(-(lp - lm) / (2 * h)) / N, float(b * b * (lp - 2 * l0 + lm) / (h * h)) / N


def moments_from_dos(dos, beta):
    """<E> and Var(E) at beta from a density of states, in mpmath."""
    b = mp.mpf(beta)
    w = {E: mp.mpf(g) * mp.exp(-b * E) for E, g in dos.items()}
    Z = mp.fsum(w.values())
    m1 = mp.fsum(E * x for E, x in w.items()) / Z
    m2 = mp.fsum(E * E * x for E, x in w.items()) / Z
    return float(m1), float(m2 - m1 * m1)
