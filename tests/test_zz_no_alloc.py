"""pd_closure_gradients_noalloc (scratch in the library's fixed device array, nothing
allocated) against pd_closure_gradients (scratch in the closure workspace) through the
C ABI: two calls in a row, the second on fewer rows, each with gradients bit for bit and
the loss within FP32 summation order (the head adds per-block partial losses with
atomics); the row limit and null outputs are rejected with an error."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pd():
    from paper_2405_08764_amd import pd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


def say(*a):
    print("[noalloc]", *a, flush=True)


def rows(n, seed):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((n, 33)) * rng.uniform(0.5, 3.0, 33)
         + rng.uniform(-2, 2, 33)).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    return torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()


def closure(pd, seed=7):
    rng = np.random.default_rng(seed)
    C = pd.Closure(max_batch=pd.NOALLOC_MAX_ROWS)
    C.set_params((0.1 * rng.standard_normal(pd.N_PARAMS)).astype(np.float32))
    X, y = rows(2048, seed + 1)
    C.fit_standardisation(X, y)
    return C


def test_noalloc_gradients_equal_workspace_gradients(pd):
    C = closure(pd)
    say("scratch bytes", pd.lib().pd_noalloc_scratch_bytes())
    grad = torch.empty(pd.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for n, seed in ((pd.NOALLOC_MAX_ROWS, 11), (1000, 12), (37, 13)):
        say("rows", n, "seed", seed)
        X, y = rows(n, seed)
        g_ref, l_ref = C.gradients(X, y)
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        C.gradients_noalloc(X, y, grad, loss)
        torch.cuda.synchronize()
        a, b = grad.cpu().numpy(), g_ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert a.tobytes() == b.tobytes(), float(np.max(np.abs(a - b)))
        la, lb = loss.item(), l_ref.item()
        # the loss is a sum of k = ceil(n / 4) non-negative block partials (one atomic add
        # per block of 4 rows) taken in any order: each FP32 add errs by at most 2^-24 of a
        # partial sum no larger than the total, so two orders differ by < 2 (k - 1) 2^-24
        bound = 2 * (-(-n // 4) - 1) * 2.0 ** -24 * abs(lb)
        say("  loss", la, lb, "bound", bound)
        assert np.isfinite(la) and abs(la - lb) <= bound


def test_noalloc_rejects_oversize_and_null(pd):
    C = closure(pd)
    grad = torch.empty(pd.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    X, y = rows(pd.NOALLOC_MAX_ROWS + 1, 3)
    with pytest.raises(pd.PdError, match="rows"):
        C.gradients_noalloc(X, y, grad, loss)
    X, y = rows(16, 4)
    with pytest.raises(pd.PdError, match="non-null"):
        C.gradients_noalloc(X, y, None, loss)
