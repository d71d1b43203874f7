"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle runs.

This module holds inputs only: lattice shapes, couplings, temperatures, seeds,
replica ids, initial-state modes and seeded +-1 arrays.  It contains none of
the method's arithmetic (no random-number stream of the sweep, no
acceptance thresholds, no update rule), so that both the GPU library and the
CPU oracle can be driven from it without sharing any of the method's code.

The paper publishes no dataset; its workloads are random-start lattices of
1024^2 to 4096^2 spins over T/J from 0.385 to 4.145 (validation, section 3.1),
2048^2 to 16384^2 single lattices (flip-rate runs, section 3.2) and up to 754
simultaneous simulations of about 200 M spins in total (section 3.2, Table 1).
The configurations below are synthetic stand-ins of those shapes.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

INIT_RANDOM, INIT_UP, INIT_DOWN = 0, 1, 2
BASE_SEED = 16990
T_CRITICAL_PRINTED = 2.269185  # critical temperature as printed in section 3.1


@dataclass
class Replica:
    Lx: int
    Ly: int
    T: float
    seed: int
    replica: int
    init: int = INIT_RANDOM
    J: float = 1.0
    rng: int = 0  # random-number contract: 0 one Philox word per site, 1 bit-sliced groups

    @property
    def beta(self) -> float:
        return 1.0 / self.T

    @property
    def spins(self) -> int:
        return self.Lx * self.Ly


@dataclass
class Workload:
    name: str
    replicas: List[Replica]
    sweeps: int
    record_every: int
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def spins(self) -> int:
        return sum(r.spins for r in self.replicas)

    @property
    def flip_attempts(self) -> int:
        return self.spins * self.sweeps


def single_64() -> Workload:
    """One 64x64 lattice at T = 2.269185, random start, 1000 sweeps, (B, M) every sweep."""
    return Workload("single-64x64-Tc", [Replica(64, 64, T_CRITICAL_PRINTED, BASE_SEED, 0)],
                    sweeps=1000, record_every=1)


def batch_256x1024() -> Workload:
    """256 replicas of 1024x1024, T_r = 1.5 + 2 r / 255, seed 16990 + r, random start."""
    reps = [Replica(1024, 1024, 1.5 + 2.0 * r / 255.0, BASE_SEED + r, r) for r in range(256)]
    return Workload("256x1024^2-T1.5..3.5", reps, sweeps=10000, record_every=100)


def uneven_512(n: int = 512) -> Workload:
    """Uneven batch: side 2^k, k uniform on {7..13}; T uniform on [2.0, 2.6).

    Both drawn from numpy's PCG64 seeded with 16990, sides first then temperatures.
    """
    rng = np.random.Generator(np.random.PCG64(BASE_SEED))
    ks = rng.integers(7, 14, size=n)
    Ts = rng.uniform(2.0, 2.6, size=n)
    reps = [Replica(1 << int(k), 1 << int(k), float(T), BASE_SEED + r, r)
            for r, (k, T) in enumerate(zip(ks, Ts))]
    return Workload("uneven-512-L128..8192", reps, sweeps=2000, record_every=100)


def paper_scale() -> Workload:
    """754 replicas of Lx=512 x Ly=528 at T = linspace(1.8, 3.0, 754), plus one
    Lx=16384 x Ly=12288 lattice at T = 2.269185; all cold (+1) starts; 1000 sweeps."""
    Ts = np.linspace(1.8, 3.0, 754)
    reps = [Replica(512, 528, float(T), BASE_SEED + r, r, INIT_UP) for r, T in enumerate(Ts)]
    reps.append(Replica(16384, 12288, T_CRITICAL_PRINTED, BASE_SEED, 754, INIT_UP))
    return Workload("paper-scale-754x512x528+16384x12288", reps, sweeps=1000, record_every=100)


# temperatures of the block-proposal workload: eight in [2.20, 2.35], one of
# them the printed critical temperature
LEARNED_TEMPS = (2.20, 2.22, 2.24, T_CRITICAL_PRINTED, 2.29, 2.31, 2.33, 2.35)
LEARNED_PER_T = 8


def learned_64x256() -> Workload:
    """64 replicas of 256x256 for the block-proposal path: 8 independent
    replicas (distinct seeds) at each temperature of LEARNED_TEMPS, replica
    r at LEARNED_TEMPS[r // 8], so an observable can be compared between two
    samplers with errors from the spread between independent replicas, and
    tau at T_c averaged over 8 chains."""
    Ts = [T for T in LEARNED_TEMPS for _ in range(LEARNED_PER_T)]
    reps = [Replica(256, 256, float(T), BASE_SEED + r, r) for r, T in enumerate(Ts)]
    return Workload("learned-64x256^2-8T-in-2.20..2.35-x8", reps, sweeps=1000, record_every=1)


@dataclass
class Replica3:
    """A 3D (simple cubic) replica."""
    Lx: int
    Ly: int
    Lz: int
    T: float
    seed: int
    replica: int
    init: int = INIT_RANDOM
    J: float = 1.0

    @property
    def beta(self) -> float:
        return 1.0 / self.T

    @property
    def spins(self) -> int:
        return self.Lx * self.Ly * self.Lz


def cubic_16x256() -> Workload:
    """16 replicas of 256^3 (the 3D generalisation of section 1), T_r = 3.5 + 2 r / 15
    around the 3D critical temperature (about 4.51), seed 16990 + r, random start."""
    reps = [Replica3(256, 256, 256, 3.5 + 2.0 * r / 15.0, BASE_SEED + r, r) for r in range(16)]
    return Workload("cubic-16x256^3-T3.5..5.5", reps, sweeps=1000, record_every=100)


ALL = {
    "single_64": single_64,
    "batch_256x1024": batch_256x1024,
    "uneven_512": uneven_512,
    "paper_scale": paper_scale,
    "learned_64x256": learned_64x256,
    "cubic_16x256": cubic_16x256,
}


def random_pm1(shape, seed: int) -> np.ndarray:
    """Seeded +-1 int8 array (numpy PCG64), for set-spins / checkpoint tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (1 - 2 * rng.integers(0, 2, size=shape)).astype(np.int8)


def small_shapes(seed: int, count: int, max_wx: int = 4, max_ly: int = 40):
    """Seeded list of (Lx, Ly) with Lx a multiple of 64 and Ly even, for parity sweeps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        out.append((64 * int(rng.integers(1, max_wx + 1)), 2 * int(rng.integers(1, max_ly // 2 + 1))))
    return out


def nn_initial_params(C: int, seed: int = 16990) -> np.ndarray:
    """Seeded initial parameters of the block-proposal network (float32, flat).

    Layout (C channels): W1[4,C], U1[4,C], v1[C], b1[C], then for layers 2..4
    W[5,C,C], b[C], then wo[C], bo[1].  Weights ~ N(0, 1/fan_in) from numpy
    PCG64(seed), biases zero.  These are inputs (random numbers drawn once),
    shared by the GPU library and the float64 reference alike.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.normal(0.0, 1.0 / np.sqrt(4.0), size=4 * C),       # W1 (4 spin taps)
             rng.normal(0.0, 1.0 / np.sqrt(4.0), size=4 * C),       # U1 (4 boundary features)
             rng.normal(0.0, 0.5, size=C),                          # v1 (beta)
             np.zeros(C)]                                           # b1
    for _ in range(3):
        parts += [rng.normal(0.0, 1.0 / np.sqrt(5.0 * C), size=5 * C * C), np.zeros(C)]
    parts += [rng.normal(0.0, 1.0 / np.sqrt(C), size=C), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)
