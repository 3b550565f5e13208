"""Pins for the adjoint, Philox/Box-Muller, BF16 rounding and the data generators."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

import genios_data
from oracle import adjoint, bf16, lasso, philox


# ---------------------------------------------------------------- adjoint --

def _fd_problem(seed):
    rng = np.random.default_rng(seed)
    m, n = 30, 50
    A = rng.standard_normal((m, n)) / np.sqrt(m) * np.arange(1, n + 1) ** -0.5
    x0 = np.zeros(n)
    x0[rng.choice(n, 4, replace=False)] = rng.standard_normal(4)
    b = A @ x0 + 0.05 * rng.standard_normal(m)
    lam = 0.1 * np.max(np.abs(A.T @ b))
    return A, b, lam, x0


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_central_differences(seed):
    A, b, lam, x0 = _fd_problem(seed)
    sol = lasso.solve(A, b, lam)
    xs = sol["x"]
    assert adjoint.strict_complementarity_margin(A, b, lam, xs) > 1e-3
    L = lambda x: float(np.sum((x - x0) ** 2))
    g = 2 * (xs - x0)
    dLdb, dLdlam, _ = adjoint.lasso_adjoint(A, xs, g)
    rng = np.random.default_rng(100 + seed)
    checked = 0
    for _ in range(6):
        d = rng.standard_normal(b.size)
        d /= np.linalg.norm(d)
        h = 1e-3
        for _ in range(4):  # halve the step while the support moves (a kink)
            sp = lasso.solve(A, b + h * d, lam)
            sm = lasso.solve(A, b - h * d, lam)
            if (np.array_equal(sp["support"], sol["support"])
                    and np.array_equal(sm["support"], sol["support"])):
                break
            h /= 2
        else:
            continue
        fd = (L(sp["x"]) - L(sm["x"])) / (2 * h)
        assert abs(fd - dLdb @ d) <= 1e-6 * max(1.0, abs(fd))
        checked += 1
    assert checked >= 3
    h = 1e-4
    sp = lasso.solve(A, b, lam * (1 + h))
    sm = lasso.solve(A, b, lam * (1 - h))
    assert np.array_equal(sp["support"], sol["support"])
    fd = (L(sp["x"]) - L(sm["x"])) / (2 * h * lam)
    assert abs(fd - dLdlam) <= 1e-6 * max(1.0, abs(fd))


# ----------------------------------------------------------------- philox --

@pytest.mark.parametrize("key", [(0, 0), (7, 11), (2 ** 64 - 1, 12345)])
def test_philox_matches_numpy(key):
    for c in (1, 2, 17, 2 ** 40):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array([c - 1, 0, 0, 0], dtype=np.uint64))
        raw = [int(v) for v in bg.random_raw(4)]
        assert list(philox.philox4x64_10((c, 0, 0, 0), key)) == raw


def test_box_muller_closed_form():
    z0, z1 = philox.normal_pair(1 << 63, 0)
    u1 = ((1 << 52) + 0.5) * 2.0 ** -53
    assert z0 == pytest.approx(math.sqrt(-2 * math.log(u1)), rel=1e-15)
    assert z1 == 0.0


def test_gaussian_matrix_distribution():
    Om = philox.gaussian_matrix(300, 40, seed=9, stream=2)
    assert Om.shape == (300, 40) and Om.dtype == np.float32
    v = Om.astype(np.float64).ravel()
    assert abs(v.mean()) < 4 / math.sqrt(v.size)
    assert abs(v.var() - 1) < 6 * math.sqrt(2 / v.size)
    assert stats.kstest(v, "norm").pvalue > 1e-3
    again = philox.gaussian_matrix(300, 40, seed=9, stream=2)
    assert np.array_equal(Om, again)
    other = philox.gaussian_matrix(300, 40, seed=9, stream=3)
    assert not np.array_equal(Om, other)


# ------------------------------------------------------------------- bf16 --

def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    vals = np.concatenate([
        rng.standard_normal(20000).astype(np.float32),
        (rng.standard_normal(2000) * 1e-40).astype(np.float32),
        (rng.standard_normal(2000) * 1e38).astype(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.4028235e38, -3.4028235e38,
                  1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9], dtype=np.float32),
        # exact ties: low 16 bits == 0x8000
        (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
    ])
    ours = bf16.round_to_bf16_bits(vals)
    ref = torch.from_numpy(vals).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    nan = np.array([np.nan, -np.nan], dtype=np.float32)
    assert np.all(np.isnan(bf16.bf16_bits_to_f32(bf16.round_to_bf16_bits(nan))))


# ------------------------------------------------------------- generators --

def test_generators_deterministic_and_shaped():
    a = genios_data.lasso_small(50, 80, 5, seed=1, s=8)
    b = genios_data.lasso_small(50, 80, 5, seed=1, s=8)
    assert np.array_equal(a["A"], b["A"]) and np.array_equal(a["b"], b["b"])
    assert a["A"].dtype == np.float32 and a["A"].flags.c_contiguous
    assert a["lam"] == pytest.approx(0.1 * np.max(np.abs(a["A"].astype(np.float64).T @ a["b"].astype(np.float64))))
    d = genios_data.lasso_decay(2100, 64, 6, seed=2, s=8)
    col = np.linalg.norm(d["A"].astype(np.float64), axis=0)
    assert col[0] > 5 * col[-1]
    lg = genios_data.logreg_factor(300, 50, seed=4, s=8)
    assert set(np.unique(lg["y"])) <= {-1.0, 1.0}
