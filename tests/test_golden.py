"""Golden fixtures: hand-derived element residuals and the paper's printed
model balance (tests/golden/*.txt carry the derivations and citations)."""
import pathlib
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1607_04245_amd import model

GOLDEN = pathlib.Path(__file__).resolve().parent / "golden"


def _cases():
    out = []
    for line in (GOLDEN / "hand_examples.txt").read_text().splitlines():
        if not line.startswith("case "):
            continue
        parts = [p.strip() for p in line[5:].split("|")]
        name = parts[0]
        dim, phys, rule = (int(v) for v in parts[1].split())
        coords = np.array(parts[2].split(), dtype=float).reshape(dim + 1, dim)
        coef = np.array(parts[3].split(), dtype=float)
        u = np.array(parts[4].split(), dtype=float)
        R = np.array(parts[5].split(), dtype=float)
        out.append((name, dim, phys, rule, coords, coef, u, R))
    return out


CASES = _cases()


def test_fixture_count():
    assert len(CASES) == 6


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_oracle_hand_examples(case):
    name, dim, phys, rule, coords, coef, u, R = case
    conn = np.arange(dim + 1, dtype=np.int32)[None]
    nq = oracle.n_qpts(dim, rule)
    got, nd = oracle.residual(dim, phys, rule, coords, conn, u[:, None], coef.reshape(-1, nq, 1))
    assert nd == 0
    assert np.allclose(got[:, 0], R, rtol=1e-14, atol=1e-15)


def test_paper_beta():
    for line in (GOLDEN / "paper_model.txt").read_text().splitlines():
        if line.startswith("#") or not line.strip():
            continue
        d, nb, nc, nq, num, den = (int(v) for v in line.split())
        assert model.paper_beta(d, nb, nc, nq) == Fraction(num, den)
        assert model.paper_flops_per_cell(d, nb, nc, nq) == 82
        assert model.paper_bytes_per_cell(d, nb, nc, nq) == 44


def test_model_counts_at_the_rules():
    # flop counts of the paper's formula at the 3- and 4-point rules
    assert model.model_flops(2, 0, 0) == 246
    assert model.model_flops(3, 0, 1) == 824
    assert model.model_flops(2, 1, 0) == 492
    assert model.model_flops(3, 1, 1) == 2472
    # compulsory words per element of the forward call
    assert [model.forward_words(*k) for k in [(2, 0, 0), (3, 0, 1), (2, 1, 0), (3, 1, 1)]] == [14, 22, 23, 42]
    assert model.backward_bytes(3, 0, 1, 4) == 120
