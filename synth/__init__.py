"""Seeded synthetic line lists, grids and conditions.

This module is the only code shared by the GPU path's tests/benchmark and the
CPU oracle.  It draws inputs and holds none of the method's arithmetic: no
line strengths, widths, profiles or k-distributions are computed here.

The paper measures on the HITRAN / HITEMP water line lists (§3, §3.5), which
are not available; these synthetic lists stand in for them, with water's mass,
a spectral span of up to 3e4 cm^-1 and 1e4 - 1e8 lines (§1.1 gives ~1e5 lines
for HITRAN water and ~1e8 for HITEMP).

Draw recipe (numpy PCG64, ``default_rng(seed)``), one full-length array per
field, in this order:
    nu        ~ U[0, nu_max)                     cm^-1
    log10 S   ~ U[-30, -18]                      S in cm/molecule at 296 K
    E''       ~ Exponential(mean 2000)           cm^-1
    gamma_air ~ U[0.02, 0.1]                     cm^-1/atm
    n_air     ~ U[0.4, 0.8]
gamma_self, delta and A21 are not drawn (absent: gamma_self = gamma_air,
delta = 0, A21 = 0).  A draw of exactly nu = 0 (probability 2^-53 per line) is
redrawn, since a line at zero wavenumber has no Doppler width.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

ATM_PER_BAR = 1.0 / 1.01325  # 1 atm = 1.01325 bar
T_REF = 296.0
MASS_H2O_AMU = 18.0


def line_list(n: int, nu_max: float, seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    nu = rng.uniform(0.0, nu_max, n)
    logS = rng.uniform(-30.0, -18.0, n)
    E = rng.exponential(2000.0, n)
    g_air = rng.uniform(0.02, 0.1, n)
    n_air = rng.uniform(0.4, 0.8, n)
    bad = nu <= 0.0
    while bad.any():
        nu[bad] = rng.uniform(0.0, nu_max, int(bad.sum()))
        bad = nu <= 0.0
    return {"nu": nu, "S_ref": 10.0 ** logS, "E_lower": E,
            "gamma_air": g_air, "n_air": n_air}


def digest(lines: dict) -> str:
    h = hashlib.sha256()
    for k in sorted(lines):
        v = lines[k]
        if v is not None:
            h.update(k.encode()); h.update(np.ascontiguousarray(v, np.float64).tobytes())
    return h.hexdigest()


def partition_ratio(T: float, T_ref: float = T_REF) -> float:
    """Q(T_ref)/Q(T) for the workloads' stated partition function
    Q(T) = Q_ref (T/296)^1.5 (an input of the workload, not of the method)."""
    return (T_ref / T) ** 1.5


def conditions(T: float, P_atm: float, mass_amu: float = MASS_H2O_AMU) -> dict:
    """Self-broadening pressure is half the total (§2.3's illustration)."""
    return {"T0": T_REF, "mass_amu": mass_amu, "T": float(T), "P": float(P_atm),
            "P_self": 0.5 * float(P_atm), "q_ratio": partition_ratio(T)}


@dataclass
class Workload:
    name: str
    n_lines: int
    nu_max: float
    dnu: float
    cutoff: float
    T: float
    P_atm: float
    n_bins: int
    n_g: int = 20
    seed: int = 0
    nu_min: float = 0.0
    states: list = field(default_factory=list)  # batched (T, P_atm) pairs

    @property
    def n_points(self) -> int:
        return int(round((self.nu_max - self.nu_min) / self.dnu))

    @property
    def points_per_bin(self) -> int:
        return self.n_points // self.n_bins

    def grid(self) -> dict:
        return {"nu_min": self.nu_min, "dnu": self.dnu, "n_points": self.n_points,
                "cutoff": self.cutoff}

    def conditions(self) -> dict:
        return conditions(self.T, self.P_atm)

    def lines(self) -> dict:
        return line_list(self.n_lines, self.nu_max, self.seed)


def _batched_states():
    Ts = np.geomspace(300.0, 3000.0, 20)
    Ps = np.geomspace(1e-6, 100.0, 10) * ATM_PER_BAR
    return [(float(T), float(P)) for T in Ts for P in Ps]


# The five workloads: CPU-sized FP64; mid-scale FP64; FP32 precision variant;
# batched (T, P) tables; learned surrogate.
WORKLOADS = {
    "lines1e4_grid3e5": Workload("lines1e4_grid3e5", 10_000, 3000.0, 0.01, 25.0,
                                 1500.0, 1.0, 3),
    "lines1e6_grid3e6": Workload("lines1e6_grid3e6", 1_000_000, 30000.0, 0.01, 100.0,
                                 1500.0, 1.0, 300),
    "lines1e7_fp32": Workload("lines1e7_fp32", 10_000_000, 30000.0, 0.01, 100.0,
                              2000.0, 0.1 * ATM_PER_BAR, 300),
    "lines1e6_tables200": Workload("lines1e6_tables200", 1_000_000, 30000.0, 0.01, 100.0,
                                   1500.0, 1.0, 300, states=_batched_states()),
    "lines1e8_surrogate": Workload("lines1e8_surrogate", 100_000_000, 30000.0, 0.01, 25.0,
                                   1500.0, 1.0, 300),
}


# ---- learned surrogate: random draws only (the method's arithmetic lives in
# the library and the oracle) ------------------------------------------------

MLP_SHAPES = [(64, 2), (64,), (64, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64,), (1,)]


def mlp_init(seed: int = 0) -> np.ndarray:
    """Initial parameters of the 2-64-64-64-64-1 network as one flat float32
    vector in the library's order (W1 b1 W2 b2 W3 b3 W4 b4 w5 b5, row-major
    W[out][in]): weights uniform on +-sqrt(6 / fan_in) (He et al. 2015),
    biases zero."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    parts = []
    for k, shape in enumerate(MLP_SHAPES):
        is_weight = k in (0, 2, 4, 6, 8)
        if is_weight:
            fan_in = shape[1] if len(shape) == 2 else shape[0]
            b = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-b, b, size=shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)


def surrogate_samples(n: int, seed: int = 0):
    """Training inputs: x uniform on [0, 50], y log-uniform on [1e-4, 1e2]
    (float32 arrays)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    x = rng.uniform(0.0, 50.0, n)
    y = 10.0 ** rng.uniform(-4.0, 2.0, n)
    return x.astype(np.float32), y.astype(np.float32)
