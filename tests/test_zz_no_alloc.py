"""hipib_spread_noalloc (spreading without a context or allocation, its node
bins in a static device workspace) against hipib_spread on an FP64 context,
through the C-ABI: two calls in a row, the second with a smaller grid and
fewer nodes, each on top of a nonzero f; plus the host-side size checks."""
import numpy as np
import pytest

from tests.test_gpu_parity import host, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def hp():
    from paper_2503_22695_amd import hipib
    hipib.lib()
    return hipib


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def spread_pair(torch, hp, n, nn, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-0.3, 1.3, (nn, 3))          # unwrapped, crossing the seam
    X[: nn // 4] = 0.5 + 0.01 * rng.standard_normal((nn // 4, 3))   # a crowded tile
    F = rng.standard_normal((nn, 3))
    f0 = rng.standard_normal((3, n, n, n))
    Xd, Fd = to_dev(torch, X), to_dev(torch, F)
    ctx = hp.Context(hp.default_config(n=n))
    ctx.set_mesh(X, np.zeros((0, 8)), np.zeros((0, 3)), np.zeros(0))
    f_ctx = to_dev(torch, f0)
    ctx.spread(Xd, Fd, f_ctx)
    f_na = to_dev(torch, f0)
    hp.spread_noalloc(n, Xd, Fd, f_na)
    torch.cuda.synchronize()
    a, b = host(f_na), host(f_ctx)
    say("spread_noalloc", n, nn, seed, rel(a, b))
    # both sum the same terms with FP64 atomics, in orders that may differ
    assert rel(a - f0, b - f0) <= 1e-13
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b - f0))


def test_spread_noalloc_matches_spread_two_calls(torch_dev, hp):
    spread_pair(torch_dev, hp, 64, 20000, 0)
    spread_pair(torch_dev, hp, 24, 3000, 1)      # smaller grid and fewer nodes


def test_spread_noalloc_rejects_sizes(torch_dev, hp):
    """Sizes beyond the workspace's limits are refused on the host, before any
    launch (status HIPIB_E_INVAL and a message naming the entry point)."""
    import ctypes as C
    torch = torch_dev
    X = torch.zeros((8, 3), dtype=torch.float64, device="cuda")
    f = torch.zeros((3, 8, 8, 8), dtype=torch.float64, device="cuda")
    p = [C.c_void_p(t.data_ptr()) for t in (X, X, f)]
    lib = hp.lib()
    for n, nn in ((512, 8), (20, 8), (4, 8), (8, (1 << 20) + 1), (8, -1)):
        st = lib.hipib_spread_noalloc(n, nn, *p, None)
        assert st == hp.E_INVAL, (n, nn, st)
        assert b"hipib_spread_noalloc" in lib.hipib_last_error()
