"""Seeded generators of the open quantum systems used as solver inputs.

This module builds Hamiltonians H and collapse operators C_k as sparse
d x d complex matrices (scipy CSR, complex128).  It holds none of the steady-
state method's arithmetic: no Liouvillian, no vectorisation, no solve.  Both
the product path (through its C ABI) and the CPU oracle consume what it makes.

Operator conventions (Fock basis for oscillators, z basis for spins, as in the
paper's numerical section):
  * a = sum_n sqrt(n) |n-1><n|   (annihilation, ones above the diagonal)
  * sigma_z = diag(1, -1); sigma_- = |1><0| (index 0 is the excited state)
  * composite operators are Kronecker products in the stated mode order.

Model families (paper section "Numerical Simulations" and the benchmark
workloads): driven Kerr oscillator, driven Jaynes-Cummings (eq. jc), driven
spin chain (eq. spinchain), optomechanics (eq. opto), a chain of coupled Kerr
cavities, and closed-form test systems (coherent, thermal, two-level atom).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np
import scipy.sparse as sp

__all__ = [
    "System", "destroy", "qeye", "sigmam", "sigmap", "sigmax", "sigmay", "sigmaz",
    "tensor", "kerr", "coherent_drive", "thermal_oscillator", "two_level_atom",
    "jaynes_cummings", "jaynes_cummings_paper", "spin_chain", "optomechanics",
    "kerr_chain", "random_lindblad", "config", "serving_stream", "CONFIG_NAMES",
]


def _csr(m) -> sp.csr_matrix:
    m = sp.csr_matrix(m, dtype=np.complex128)
    m.eliminate_zeros()
    m.sum_duplicates()
    m.sort_indices()
    return m


def destroy(n: int) -> sp.csr_matrix:
    """Annihilation operator in an n-state Fock basis."""
    return _csr(sp.diags(np.sqrt(np.arange(1, n, dtype=np.float64)), 1, shape=(n, n)))


def qeye(n: int) -> sp.csr_matrix:
    return _csr(sp.identity(n, dtype=np.complex128, format="csr"))


def sigmam() -> sp.csr_matrix:
    return _csr(np.array([[0, 0], [1, 0]], dtype=np.complex128))


def sigmap() -> sp.csr_matrix:
    return _csr(np.array([[0, 1], [0, 0]], dtype=np.complex128))


def sigmax() -> sp.csr_matrix:
    return _csr(np.array([[0, 1], [1, 0]], dtype=np.complex128))


def sigmay() -> sp.csr_matrix:
    return _csr(np.array([[0, -1j], [1j, 0]], dtype=np.complex128))


def sigmaz() -> sp.csr_matrix:
    return _csr(np.array([[1, 0], [0, -1]], dtype=np.complex128))


def tensor(*ops) -> sp.csr_matrix:
    """Kronecker product of operators in the order given (first = leftmost)."""
    out = ops[0]
    for o in ops[1:]:
        out = sp.kron(out, o, format="csr")
    return _csr(out)


def dag(m: sp.csr_matrix) -> sp.csr_matrix:
    return _csr(m.conj().T)


@dataclass
class System:
    """An open system: Hamiltonian and collapse operators, plus metadata."""
    name: str
    H: sp.csr_matrix
    c_ops: List[sp.csr_matrix]
    params: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return self.H.shape[0]


# --------------------------------------------------------------------------
# single-mode systems
# --------------------------------------------------------------------------
def kerr(N: int = 20, delta: float = 0.5, chi: float = 0.1, E: float = 1.0,
         kappa: float = 1.0) -> System:
    """Driven damped Kerr oscillator: H = D a+a + (chi/2) a+a+aa + E(a + a+),
    one collapse operator sqrt(kappa) a."""
    a = destroy(N)
    ad = dag(a)
    H = delta * (ad @ a) + 0.5 * chi * (ad @ ad @ a @ a) + E * (a + ad)
    return System(f"kerr_N{N}", _csr(H), [_csr(np.sqrt(kappa) * a)],
                  dict(N=N, delta=delta, chi=chi, E=E, kappa=kappa))


def coherent_drive(N: int = 40, delta: float = 0.5, E: float = 1.0,
                   kappa: float = 1.0) -> System:
    """Linear driven damped cavity (Kerr term off); its steady state is the
    coherent state with alpha = -iE/(kappa/2 + i delta)."""
    s = kerr(N, delta, 0.0, E, kappa)
    s.name = f"coherent_N{N}"
    return s


def thermal_oscillator(N: int = 20, nbar: float = 2.0, kappa: float = 1.0,
                       omega: float = 1.0) -> System:
    """Oscillator coupled to a thermal bath: C1 = sqrt(kappa(1+n)) a,
    C2 = sqrt(kappa n) a+, H = omega a+a."""
    a = destroy(N)
    ad = dag(a)
    return System(f"thermal_N{N}", _csr(omega * (ad @ a)),
                  [_csr(np.sqrt(kappa * (1 + nbar)) * a), _csr(np.sqrt(kappa * nbar) * ad)],
                  dict(N=N, nbar=nbar, kappa=kappa, omega=omega))


def two_level_atom(delta: float = 0.3, omega_rabi: float = 0.7, gamma: float = 0.5) -> System:
    """Driven two-level atom: H = delta s+s- + (Omega/2) sx, C = sqrt(gamma) s-."""
    sm = sigmam()
    H = delta * (dag(sm) @ sm) + 0.5 * omega_rabi * sigmax()
    return System("two_level", _csr(H), [_csr(np.sqrt(gamma) * sm)],
                  dict(delta=delta, omega_rabi=omega_rabi, gamma=gamma))


# --------------------------------------------------------------------------
# the paper's model families
# --------------------------------------------------------------------------
def _jc_hamiltonian(a, sm, delta, omega_a, g, E):
    # eq. (jc): H = -D a+a + w_a s+s- + g (a + a+)(s- + s+) + E (a + a+)
    ad, sp_ = dag(a), dag(sm)
    return -delta * (ad @ a) + omega_a * (sp_ @ sm) + g * ((a + ad) @ (sm + sp_)) + E * (a + ad)


def jaynes_cummings(N: int = 40, seed: int = 0) -> System:
    """Driven Jaynes-Cummings, cavity (N states) x qubit, parameters
    (g, E, Delta_c, omega_a, kappa, gamma) drawn in that order from a seeded
    uniform [0.1, 2]; collapse sqrt(kappa) a and sqrt(gamma) s-."""
    g, E, delta, omega_a, kappa, gamma = np.random.default_rng(seed).uniform(0.1, 2.0, 6)
    a = tensor(destroy(N), qeye(2))
    sm = tensor(qeye(N), sigmam())
    H = _jc_hamiltonian(a, sm, delta, omega_a, g, E)
    c_ops = [_csr(np.sqrt(kappa) * a), _csr(np.sqrt(gamma) * sm)]
    return System(f"jc_N{N}", _csr(H), c_ops,
                  dict(N=N, g=g, E=E, delta=delta, omega_a=omega_a, kappa=kappa,
                       gamma=gamma, seed=seed))


def jaynes_cummings_paper(N: int = 16, delta: float = 0.0, omega_a: float = 1.0,
                          g: float = 0.25, E: float = 1.0, kappa: float = 5e-3,
                          gamma: float = 0.05, nth: float = 1.0) -> System:
    """The paper's Jaynes-Cummings system (eq. jc) with its thermal collapse set
    and operator order s- = s- x I, a = I x a."""
    sm = tensor(sigmam(), qeye(N))
    a = tensor(qeye(2), destroy(N))
    H = _jc_hamiltonian(a, sm, delta, omega_a, g, E)
    c_ops = [_csr(np.sqrt(kappa * (1 + nth)) * a), _csr(np.sqrt(kappa * nth) * dag(a)),
             _csr(np.sqrt(gamma * (1 + nth)) * sm)]
    return System(f"jc_paper_N{N}", _csr(H), c_ops,
                  dict(N=N, delta=delta, omega_a=omega_a, g=g, E=E, kappa=kappa,
                       gamma=gamma, nth=nth))


def spin_chain(N: int = 5, omega: float = 2 * np.pi, J: float = 0.1 * 2 * np.pi,
               detuning: float = 0.0, gamma: float = 0.01) -> System:
    """Driven spin chain, eq. (spinchain): first spin driven with Omega = omega/2,
    identical spin frequencies, isotropic nearest-neighbour couplings J, and
    dephasing sqrt(gamma) s_z on every spin.  The drive detuning is not given
    numerically; 0 (resonant drive) is used."""
    def op(single, k):
        return tensor(*[single if i == k else qeye(2) for i in range(N)])
    sx = [op(sigmax(), k) for k in range(N)]
    sy = [op(sigmay(), k) for k in range(N)]
    sz = [op(sigmaz(), k) for k in range(N)]
    rabi = omega / 2
    H = -0.5 * detuning * sz[0] - 0.5 * rabi * sx[0]
    for n in range(1, N):
        H = H - 0.5 * omega * sz[n]
    for n in range(N - 1):
        H = H - 0.5 * (J * sx[n] @ sx[n + 1] + J * sy[n] @ sy[n + 1] + J * sz[n] @ sz[n + 1])
    c_ops = [_csr(np.sqrt(gamma) * sz[n]) for n in range(N)]
    return System(f"spin_chain_{N}", _csr(H), c_ops,
                  dict(N=N, omega=omega, J=J, detuning=detuning, gamma=gamma))


def optomechanics(Nc: int = 10, Nm: int = 60, delta: float = 0.0, omega_m: float = 1.0,
                  g0: float = 0.4, E: float = 0.1, kappa: float = 0.3,
                  gamma: float = 1e-4, nth: float = 2.0) -> System:
    """Optomechanics, eq. (opto): H = -D a+a + w_m b+b + g0 (b + b+) a+a + E(a + a+),
    order a x I, I x b; collapse sqrt(kappa) a, sqrt(gamma(1+n)) b, sqrt(gamma n) b+."""
    a = tensor(destroy(Nc), qeye(Nm))
    b = tensor(qeye(Nc), destroy(Nm))
    ad, bd = dag(a), dag(b)
    H = -delta * (ad @ a) + omega_m * (bd @ b) + g0 * ((b + bd) @ (ad @ a)) + E * (a + ad)
    c_ops = [_csr(np.sqrt(kappa) * a)]
    if gamma * (1 + nth) != 0:
        c_ops.append(_csr(np.sqrt(gamma * (1 + nth)) * b))
    if gamma * nth != 0:
        c_ops.append(_csr(np.sqrt(gamma * nth) * bd))
    return System(f"optomech_{Nc}x{Nm}", _csr(H), c_ops,
                  dict(Nc=Nc, Nm=Nm, delta=delta, omega_m=omega_m, g0=g0, E=E,
                       kappa=kappa, gamma=gamma, nth=nth))


def kerr_chain(sites: int = 3, N: int = 10, delta: float = 0.5, chi: float = 0.1,
               E: float = 1.0, kappa: float = 1.0, J: float = 0.3) -> System:
    """Chain of coupled driven Kerr cavities, order site1 x site2 x ...;
    per-site Kerr Hamiltonian and loss sqrt(kappa) a_i, hopping
    J (a_i+ a_{i+1} + h.c.)."""
    def op(single, k):
        return tensor(*[single if i == k else qeye(N) for i in range(sites)])
    a = [op(destroy(N), k) for k in range(sites)]
    ad = [dag(x) for x in a]
    H = None
    for k in range(sites):
        hk = delta * (ad[k] @ a[k]) + 0.5 * chi * (ad[k] @ ad[k] @ a[k] @ a[k]) + E * (a[k] + ad[k])
        H = hk if H is None else H + hk
    for k in range(sites - 1):
        if J != 0:
            H = H + J * (ad[k] @ a[k + 1] + ad[k + 1] @ a[k])
    c_ops = [_csr(np.sqrt(kappa) * a[k]) for k in range(sites)]
    return System(f"kerr_chain_{sites}x{N}", _csr(H), c_ops,
                  dict(sites=sites, N=N, delta=delta, chi=chi, E=E, kappa=kappa, J=J))


def random_lindblad(d: int, n_cops: int = 2, density: float = 0.5, seed: int = 0) -> System:
    """Random Hermitian H and random sparse collapse operators (generic: unique
    steady state with probability one)."""
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    mask = rng.random((d, d)) < density
    A = np.where(mask | mask.T, A, 0)
    H = 0.5 * (A + A.conj().T)
    c_ops = []
    for _ in range(n_cops):
        C = (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))) * (rng.random((d, d)) < density)
        C[np.arange(d - 1) + 1, np.arange(d - 1)] += 1.0  # a lowering ladder keeps it ergodic
        c_ops.append(_csr(0.5 * C))
    return System(f"random_d{d}_s{seed}", _csr(H), c_ops, dict(d=d, n_cops=n_cops, seed=seed))


# --------------------------------------------------------------------------
# benchmark workloads
# --------------------------------------------------------------------------
CONFIG_NAMES = {
    1: "kerr_N20",
    2: "jc_N40xqubit",
    3: "optomech_10x60_nth2",
    4: "kerr_chain_3x10",
    5: "serving_kerr_N10to60",
}


def config(k: int) -> System:
    """The solver workloads 1..4 (5 is a request stream, see serving_stream)."""
    if k == 1:
        return kerr(20, 0.5, 0.1, 1.0, 1.0)
    if k == 2:
        return jaynes_cummings(40, seed=0)
    if k == 3:
        return optomechanics(10, 60, nth=2.0)
    if k == 4:
        return kerr_chain(3, 10, J=0.3)
    raise ValueError(f"no system config {k}")


def serving_stream(n_requests: int = 2000, rate: float = 1.0, seed: int = 1,
                   n_min: int = 10, n_max: int = 60):
    """Request stream of Kerr steady-state problems: cutoff N ~ U{n_min..n_max},
    (Delta, E) drawn from a 21 x 20 sweep grid, chi = 0.1, kappa = 1; arrival
    times from a Poisson process of the given rate (requests per second).
    Returns a list of (arrival_time_s, N, delta, E)."""
    rng = np.random.default_rng(seed)
    deltas = np.linspace(-1.0, 1.0, 21)
    Es = np.linspace(0.1, 2.0, 20)
    Ns = rng.integers(n_min, n_max + 1, size=n_requests)
    di = rng.integers(0, len(deltas), size=n_requests)
    ei = rng.integers(0, len(Es), size=n_requests)
    gaps = rng.exponential(1.0 / rate, size=n_requests) if rate > 0 else np.zeros(n_requests)
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[i]), int(Ns[i]), float(deltas[di[i]]), float(Es[ei[i]])) for i in range(n_requests)]
