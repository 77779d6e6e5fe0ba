"""The algorithmic byte and flop model against the numbers the paper prints."""
import os

import pytest

from paper_1803_02156_amd import traffic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kv(name):
    out, rows = {}, []
    for line in open(os.path.join(GOLD, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        parts = line.split()
        if len(parts) == 2:
            out[parts[0]] = float(parts[1])
        else:
            rows.append(tuple(float(p) for p in parts))
    return out, rows


def test_table3_minimum_volume():
    kv, _ = _kv("paper_table3_minimum_traffic.txt")
    n, nb = int(kv["n"]), int(kv["n_b"])
    r, w = traffic.step_bytes(n, int(kv["nnzr"]) * n, nb, prec=0)
    assert round(r / 1e9, 2) == kv["read_GB"]
    assert round(w / 1e9, 2) == kv["write_GB"]


def test_eq2_intensity_and_roofline():
    kv, rows = _kv("paper_eq2_roofline.txt")
    assert traffic.intensity(4) == pytest.approx(146 / (260 / 4 + 80))
    # limit 146/80 = 1.825, printed rounded up as 1.83
    assert abs(146 / 80 - kv["intensity_limit"]) <= 0.005 + 1e-12
    assert traffic.intensity(10 ** 12) == pytest.approx(146 / 80, rel=1e-9)
    for b, nb, pstar in rows:
        # the paper rounds 543.7 -> 540, 961.1 -> 960, 473.2 -> 470, 836.5 -> 836
        assert abs(traffic.roofline(int(nb), b) - pstar) / pstar < 0.01


def test_mixed_bytes_halve_vectors():
    n, nb = 1000, 32
    r64, w64 = traffic.step_bytes(n, 13 * n, nb, 0)
    r32, w32 = traffic.step_bytes(n, 13 * n, nb, 1)
    assert (r64 + w64) / n == 260 + 80 * nb
    assert (r32 + w32) / n == 156 + 40 * nb
