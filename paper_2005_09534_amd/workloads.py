"""Seeded synthetic workloads: the disordered spin chains the paper studies.

This module only draws inputs (random fields h_i, start-block seeds) and names
the configurations; it holds none of the method's arithmetic, so both the GPU
path and the CPU oracle can be fed from it.

Fields are i.i.d. uniform on [-W, W] (paper, "Benchmark models"), J1 = 1 and
periodic boundary conditions throughout.  The target is the rescaled energy
eps = 0.5 (the middle of the spectrum, sigma = 0 in H~ units, as in every
benchmark of the paper).
"""

from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class Chain:
    L: int
    J1: float
    J2: float
    Delta: float
    h: np.ndarray
    W: float = 0.0
    seed: int = 0


@dataclass
class Workload:
    name: str
    chains: List[Chain]
    nev: int
    block: int          # 0 = autotuned
    precision: str      # "fp64" or "fp32"
    K: int = 0          # 0 = chosen from the density of states
    eps_target: float = 0.5
    note: str = ""
    extra: dict = field(default_factory=dict)


def fields(L, W, seed):
    """h_i ~ U[-W, W], i = 1..L, FP64, from numpy's default generator."""
    return np.random.default_rng(seed).uniform(-W, W, L)


def chain(L, W, seed, J1=1.0, J2=0.0, Delta=1.0):
    return Chain(L=L, J1=J1, J2=J2, Delta=Delta, h=fields(L, W, seed), W=W, seed=seed)


def c1():
    """L=12 XXZ, W=3, N_ev=20, s=4, K=200, FP64 (dense-checkable)."""
    return Workload("xxz_L12_W3_nev20_s4_K200_fp64", [chain(12, 3.0, 1)], nev=20, block=4,
                    precision="fp64", K=200)


def c2():
    """L=18 J1-J2 (J2=1, Delta=1), W=2, N_ev=50, s=16, K auto, FP64."""
    return Workload("j1j2_L18_W2_nev50_s16_fp64", [chain(18, 2.0, 2, J2=1.0, Delta=1.0)],
                    nev=50, block=16, precision="fp64")


def c3(precision="fp32"):
    """L=22 XXZ, W=5, N_ev=100, s=32; FP32 filter vs all-FP64 on one seed."""
    return Workload(f"xxz_L22_W5_nev100_s32_{precision}", [chain(22, 5.0, 3)], nev=100, block=32,
                    precision=precision)


def c4(R=512):
    """R realisations, L_r = (14, 16, 18)[r mod 3], W_r = 1 + floor(r/3) mod 5,
    N_ev = 20 each, FP32 filter, block size autotuned."""
    chains = []
    for r in range(R):
        L = (14, 16, 18)[r % 3]
        W = float(1 + (r // 3) % 5)
        chains.append(chain(L, W, 1000 + r))
    return Workload(f"xxz_batch{R}_L14-16-18_W1-5_nev20_fp32", chains, nev=20, block=0,
                    precision="fp32")


def c5():
    """L=26 XXZ, W=4, N_ev=100, s=64, FP32 filter + FP64 Rayleigh-Ritz."""
    return Workload("xxz_L26_W4_nev100_s64_fp32", [chain(26, 4.0, 5)], nev=100, block=64,
                    precision="fp32")


def j1j2_paper(L, nev, precision="fp64", W=4.0, seed=7):
    """The paper's J1-J2 benchmark model (J2 = 1, Delta = 0.55; main text,
    "Benchmark models") at the sizes of its J1-J2 timing table (Supplement,
    "Benchmark for disorder spin chains": L = 20 with N_ev = 100, 1000 and
    L = 22 with N_ev = 100, 200, 1400, all at the middle of the spectrum).
    The table does not state the disorder strength; W = 4 stands in for it.
    Block size 16 (FP64) or 32 (FP32)."""
    return Workload(f"j1j2_L{L}_D0.55_W{W:g}_nev{nev}_{precision}",
                    [chain(L, W, seed, J2=1.0, Delta=0.55)], nev=nev,
                    block=16 if precision == "fp64" else 32, precision=precision)


def random_block(n, s, seed):
    """Seeded N(0,1) block (n x s), FP64, row-major: a test input."""
    return np.random.default_rng(seed).standard_normal((n, s))
