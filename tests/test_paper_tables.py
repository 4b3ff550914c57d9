"""The cost arithmetic printed in the paper's Tables 1-2 (values in tests/golden).

Pins the cost model used when reporting work per survey: O(Nx Nr^2 Nt^3) for the
direct Toeplitz products, O(Nx Nr^2 Nt^2) for the Fourier-diagonal build, and
2 PDE solves per CG/GMRES iteration per source.
"""
import json
import os

import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _rel(a, b):
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("row", GOLD["table1"], ids=lambda r: r["model"])
def test_table1_operation_counts(row):
    nx = row["nx"][0] * row["nx"][1]
    direct = nx * row["nr"] ** 2 * row["nt"] ** 3
    proposed = nx * row["nr"] ** 2 * row["nt"] ** 2
    rd = row["randomized_dims"]
    randomized = rd["nx"][0] * rd["nx"][1] * rd["nr"] ** 2 * rd["nt"] ** 2
    assert _rel(direct, row["direct"]) < 5e-3
    assert _rel(proposed, row["proposed"]) < 5e-3
    assert _rel(randomized, row["randomized"]) < 5e-3
    assert _rel(direct / randomized, row["speedup"]) < 0.05


@pytest.mark.parametrize("row", GOLD["table2"], ids=lambda r: r["model"])
def test_table2_pde_counts(row):
    assert row["cg"] == 2 * row["cg_iters"] * row["sources"]
    assert row["gmres"] == 2 * row["gmres_iters"] * row["sources"]


@pytest.mark.parametrize("row", GOLD["receiver_gains"], ids=lambda r: f'{r["from"]}->{r["to"]}')
def test_receiver_gain_is_quadratic(row):
    assert _rel((row["from"] / row["to"]) ** 2, row["gain"]) < 2e-3
