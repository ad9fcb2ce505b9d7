"""The paper's workload and latency model (Table 1, Table 2, Tables 4-5).

TEST INFRASTRUCTURE ONLY (pins the paper's own accounting; the tests check
it against the theoretical-latency columns of Tables 4 and 5).

Conventions, from the paper:
* one complex multiply = 6 operations; with the accumulation of a direct
  FIR tap, 8 (Section 3.3 and the 8NKM requirement of Section 3);
* an N_FT-point FFT costs C * N_FT * log2(N_FT) with C = 5 for the FFT
  engine used (Section 4.2);
* a direct/OLA TD kernel streams one input point per clock per launch and is
  launched R = ceil(K / K') times per filter (Section 4.1, Table 2);
* an OLS-FD launch takes ceil(N / (N_FT - K)) * N_FT / N_FT_PC clocks
  (Section 5.2.3); AOLS runs the engine twice per filter (FFT round, then
  multiply+IFFT round), TOLS once.
"""
from __future__ import annotations

import math


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


# --- Table 1: operation counts -------------------------------------------

def td_naive_ops(n: int, k: int) -> float:
    return 8.0 * k * n


def td_ola_ops(n: int, k: int, k_sub: int) -> float:
    return 8.0 * k_sub * n * ceil_div(k, k_sub)


def fd_naive_ops(n: int, c: float = 5.0, averaged: bool = False) -> float:
    return n * (6.0 + (1.0 if averaged else 2.0) * c * math.log2(n))


def fd_ols_ops(n: int, k: int, n_ft: int, c: float = 5.0, averaged: bool = False) -> float:
    return ceil_div(n, n_ft - k) * n_ft * (6.0 + (1.0 if averaged else 2.0) * c * math.log2(n_ft))


# --- Section 3: real-time requirement -------------------------------------

INTEGRATION_S = 536.87
DM_TRIALS = 6000


def t_limit_s() -> float:
    """Time available per DM trial: integration time / number of DM trials."""
    return INTEGRATION_S / DM_TRIALS


def required_flops(n: int = 1 << 22, k: int = 421, m: int = 84) -> float:
    """8 N K M / t_limit: direct-convolution rate needed for one beam."""
    return 8.0 * n * k * m / t_limit_s()


# --- Table 2: kernel launches ---------------------------------------------

def launches(kind: str, m: int, r: int = 1) -> int:
    kind = kind.lower()
    if kind in ("td-naive", "td-ola"):
        return r * m
    if kind in ("fd-naive", "aols"):
        return m + 1 if m > 1 else 2
    if kind == "tols":
        return m
    raise ValueError(kind)


# --- Tables 4 and 5: theoretical latency ----------------------------------

def td_latency_s(n: int, k: int, fmax_hz: float, k_sub: int = 64) -> float:
    """R * N clocks for a K-tap filter on a K'-wide TD structure."""
    return ceil_div(k, k_sub) * n / fmax_hz


def ols_launch_cycles(n: int, k: int, n_ft: int, n_ft_pc: int) -> int:
    return ceil_div(n, n_ft - k) * (n_ft // n_ft_pc)


def ols_latency_s(n: int, k: int, n_ft: int, fmax_hz: float, kind: str = "aols",
                  n_ft_pc: int = 8) -> float:
    """Single filter: AOLS runs the engine twice, TOLS once."""
    rounds = 2 if kind.lower() == "aols" else 1
    return rounds * ols_launch_cycles(n, k, n_ft, n_ft_pc) / fmax_hz


def ols_power_avg_latency_s(n: int, k: int, n_ft: int, fmax_hz: float, replicas: int,
                            n_ft_pc: int = 4) -> float:
    """Average per-filter latency of `replicas` AOLS-N_FT-P structures working on
    different filters (forward round amortised away over many filters)."""
    return ols_launch_cycles(n, k, n_ft, n_ft_pc) / (replicas * fmax_hz)
