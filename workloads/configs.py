"""The five benchmark workloads as seeded generator recipes.

Each recipe names the grid, viscosity, stretching, wind, number of subdomains,
aggregate size, Krylov settings and the storage precisions of the
preconditioner factors.  Seeds: 1001, 1002, 1003 and 1005 for the four
single systems, 4000 + s for system s of the batched workload, 5000 + t for
learned-model training instance t.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .mac_oseen import Wind, make_oseen_mac

F64, F32, F16_SCALED, BF16 = 0, 1, 2, 3


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    nu: float
    stretch: float | None
    m: int
    sz: int
    restart: int
    flexible: bool
    tol: float
    seed: int
    interior_prec: int
    schur_prec: int
    wind_coeffs: tuple = (1.0, 0.0, 0.0, 0.0)
    wind_scale: float = 1.0
    scheme: str = "central"

    def build(self):
        w = Wind(self.wind_coeffs, self.wind_scale)
        return make_oseen_mac(self.n, self.nu, wind=w, stretch=self.stretch, seed=self.seed, scheme=self.scheme)


CAVITY16 = Workload("cavity16_uniform_nu0.1_m4", 16, 1 / 10, None, 4, 64, 30, False, 1e-8, 1001, F64, F64)
CAVITY128 = Workload("cavity128_uniform_nu0.01_m16", 128, 1 / 100, None, 16, 64, 50, True, 1e-8, 1002, F32, F32)
CAVITY256_STRETCHED = Workload("cavity256_stretched1.05_nu0.001_m64", 256, 1 / 1000, 1.05, 64, 64, 50, True, 1e-8, 1003,
                F32, F16_SCALED)
CAVITY512_STRETCHED = Workload("cavity512_stretched1.05_nu0.002_m256", 512, 1 / 500, 1.05, 256, 64, 50, True, 1e-8, 1005,
                F32, F32)

WORKLOADS = {w.name: w for w in (CAVITY16, CAVITY128, CAVITY256_STRETCHED, CAVITY512_STRETCHED)}


def batched_workloads(count: int = 96, base_seed: int = 4000):
    """Independent systems of the batched workload: n ~ U{32..128} (even),
    nu log-uniform in [1/500, 1/20], a random combination of the four
    recirculating wind modes scaled to max |w| = 2, m ~ U{4..16}."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(base_seed + s)
        n = int(rng.integers(16, 65)) * 2
        nu = float(np.exp(rng.uniform(np.log(1 / 500), np.log(1 / 20))))
        w = Wind.random_modes(rng)
        m = int(rng.integers(4, 17))
        out.append(Workload(f"batch{s}_n{n}", n, nu, None, m, 64, 50, True, 1e-8, base_seed + s,
                            F32, F32, w.c, w.s))
    return out


def training_workloads(count: int = 2000, base_seed: int = 5000):
    """Instances for the learned interface correction: 64 x 64 cells, nu
    log-uniform in [1/1000, 1/20], a random combination of the four wind
    modes scaled to max |w| = 2, a uniform grid or a geometric stretching of
    ratio U(1.01, 1.08), m = 4 subdomains, aggregates of 64."""
    out = []
    for t in range(count):
        rng = np.random.default_rng(base_seed + t)
        nu = float(np.exp(rng.uniform(np.log(1 / 1000), np.log(1 / 20))))
        w = Wind.random_modes(rng)
        st = None if rng.random() < 0.5 else float(rng.uniform(1.01, 1.08))
        out.append(Workload(f"train{t}", 64, nu, st, 4, 64, 50, True, 1e-8, base_seed + t,
                            F32, F32, w.c, w.s))
    return out
