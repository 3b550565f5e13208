"""genios_hvp_noalloc (the H p product without a workspace) against genios_hvp."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def g():
    import paper_2310_08333_amd as g
    return g


def _case(g, m, n, bf16, weighted, seed):
    rng = np.random.default_rng(seed)
    A = torch.from_numpy(rng.standard_normal((m, n)).astype(np.float32)).to(DEV)
    A16 = g.cast_bf16(A) if bf16 else None
    p = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(DEV)
    d = (torch.from_numpy(rng.uniform(0.0, 0.25, m).astype(np.float32)).to(DEV)
         if weighted else None)
    return A, A16, p, d


# Two calls in a row on one GPU, the second on a smaller input: the scratch buffer
# keeps the first call's partial sums, which the second must not pick up.
SEQUENCES = [
    [(4096, 8192, True, False), (1000, 1000, True, True)],
    [(3000, 4104, False, True), (513, 1003, False, False)],
]


@pytest.mark.parametrize("seq", SEQUENCES, ids=["bf16", "fp32"])
def test_hvp_noalloc_equals_hvp(g, seq):
    for k, (m, n, bf16, weighted) in enumerate(seq):
        print("hvp_noalloc", k, m, n, "bf16" if bf16 else "fp32", "d" if weighted else "-",
              flush=True)
        A, A16, p, d = _case(g, m, n, bf16, weighted, seed=100 + k)
        ref = g.hvp(A, p, d=d, A16=A16)
        out = torch.full_like(ref, float("nan"))
        got = g.hvp_noalloc(A, p, d=d, A16=A16, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        # same kernels, same launch shapes, fixed-order reductions: bitwise equal
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), (m, n)
        # and the product itself, against FP64 on the same (rounded) entries
        A64 = (A16.view(torch.bfloat16).float() if bf16 else A).double().cpu().numpy()
        dd = np.ones(m) if d is None else d.double().cpu().numpy()
        pp = p.double().cpu().numpy()
        exact = A64.T @ (dd * (A64 @ pp))
        bound = (m + n + 520) * 2.0 ** -24 * (np.abs(A64).T @ (dd * (np.abs(A64) @ np.abs(pp))))
        assert np.all(np.abs(got.double().cpu().numpy() - exact) <= bound + 1e-30)
