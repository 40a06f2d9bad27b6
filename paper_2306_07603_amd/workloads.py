"""Seeded synthetic workloads: cavity parameter sets only (no arithmetic of the method).

Shared by the tests, the smoke check and the benchmark, and used to feed the
same inputs to the GPU library and to the CPU oracle.  Every workload is the
paper's lid-driven problem (Section 2): fluid at rest, lid at u0 = 0.1, CFL
0.5 (Section 5), with the cavity sizes, Reynolds numbers, power-law indices
and top angles of the study (Sections 5-6) drawn or listed below.
"""
from __future__ import annotations

from dataclasses import dataclass

MASK64 = (1 << 64) - 1


def splitmix64(state: int):
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def uniforms(seed: int, count: int):
    """count doubles in [0, 1) from SplitMix64 seeded with `seed` (53 high bits each)."""
    out, s = [], seed & MASK64
    for _ in range(count):
        s, z = splitmix64(s)
        out.append((z >> 11) * (1.0 / (1 << 53)))
    return out


@dataclass(frozen=True)
class CavitySpec:
    n_xi: int
    n_eta: int
    re: float
    n: float
    theta_deg: float
    u_lid: float = 0.1


def single_small():
    """33 x 33 nodes, theta = 60 deg, n = 0.8, Re = 100: the 2000-step FP64 parity case."""
    return CavitySpec(33, 33, 100.0, 0.8, 60.0)


def precision_sweep():
    """257 x 257 nodes at Re = 1000 for n in {0.5, 1, 1.5} and theta in {45, 60, 90} deg."""
    return [CavitySpec(257, 257, 1000.0, n, th) for n in (0.5, 1.0, 1.5) for th in (45.0, 60.0, 90.0)]


BATCH_SIDES = (65, 129, 257, 513)


def batch_sweep(count: int = 256):
    """The uneven batch: cavity c draws r1..r4 from SplitMix64 seeded with c;
    side = {65, 129, 257, 513}[floor(4 r1)], Re = 100 * 50^r2 (log-uniform in
    [100, 5000]), n = 0.5 + r3, theta = 40 + 50 r4 deg, lid speed 0.1."""
    out = []
    for c in range(count):
        r1, r2, r3, r4 = uniforms(c, 4)
        side = BATCH_SIDES[min(int(4 * r1), 3)]
        out.append(CavitySpec(side, side, 100.0 * 50.0 ** r2, 0.5 + r3, 40.0 + 50.0 * r4))
    return out


def adjoint_case():
    """129 x 129 nodes, theta = 60 deg, n = 0.7, Re = 400."""
    return CavitySpec(129, 129, 400.0, 0.7, 60.0)


def large_unsteady():
    """1025 x 1025 nodes, theta = 75 deg, n = 1.2, Re = 10^4."""
    return CavitySpec(1025, 1025, 1.0e4, 1.2, 75.0)
