"""The paper's workload model against the numbers it prints (Tables 4 and 5,
and the real-time requirement of Section 3)."""
import os

import pytest

from oracle import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
N = 1 << 22
K = 421


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _table4():
    return [(r[0], float(r[1]), float(r[2])) for r in _rows("table4_theoretical_latency.txt")]


@pytest.mark.parametrize("name,fmax,lat_ms", _table4())
def test_table4_theoretical_latency(name, fmax, lat_ms):
    if name.startswith(("TD", "OLA")):
        got = workload.td_latency_s(N, K, fmax * 1e6, k_sub=64) * 1e3
    else:
        kind, n_ft = name.split("-")
        got = workload.ols_latency_s(N, K, int(n_ft), fmax * 1e6, kind=kind, n_ft_pc=8) * 1e3
    assert abs(got - lat_ms) / lat_ms <= 0.005, (name, got, lat_ms)


def test_table5_power_kernels():
    for name, reps, fmax, lat_ms, fits in _rows("table5_power_kernels.txt"):
        n_ft = int(name.split("-")[1])
        got = workload.ols_power_avg_latency_s(N, K, n_ft, float(fmax) * 1e6, int(reps)) * 1e3
        err = abs(got - float(lat_ms)) / float(lat_ms)
        if fits == "1":
            assert err <= 0.005, (name, reps, got, lat_ms)
        else:
            # printed value is ~1.42x the cycle formula; recorded, not reproduced
            assert 1.35 < float(lat_ms) / got < 1.5


def test_realtime_requirement():
    vals = dict((r[0], float(r[1])) for r in _rows("realtime_requirement.txt"))
    assert abs(workload.t_limit_s() * 1e3 - vals["t_limit_ms"]) < 0.05
    assert abs(workload.required_flops() / 1e12 - vals["required_tflops"]) < 0.01
    assert workload.required_flops() * vals["beams"] / 1e15 > vals["required_pflops_all_beams"]


def test_table1_identities():
    # OLA equals naive when K' divides K; FD averaged form is below single form
    assert workload.td_ola_ops(N, 448, 64) == workload.td_naive_ops(N, 448)
    assert workload.td_ola_ops(N, 421, 64) > workload.td_naive_ops(N, 421)
    assert workload.fd_ols_ops(N, K, 2048, averaged=True) < workload.fd_ols_ops(N, K, 2048)
    assert workload.launches("aols", 84) == 85 and workload.launches("tols", 84) == 84
    assert workload.launches("td-ola", 84, r=7) == 588
