"""The allocation-free network forward (pmg_net_forward_noalloc) against
pmg_net_forward, through the C-ABI.

Both run the same GEMM kernels on the same rows (every output row depends on
its own input row only, so the chunking does not change the arithmetic): the
outputs must be equal bit for bit.  Two calls in a row, the second on fewer
rows than the first, check that nothing the first call left in the shared
activation array leaks into the second.
"""
import numpy as np
import pytest

from gpu_common import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2009_00705_amd import pmg
    from paper_2009_00705_amd import workloads as W
    c = pmg.Context(W.box_mesh(3, 2), P=4)
    yield c
    c.close()


def _inputs(n, seed):
    return np.random.default_rng(seed).standard_normal((n, 7)).astype(np.float32)


@pytest.mark.parametrize("width,depth", [(160, 3), (256, 2), (32, 0)])
def test_noalloc_forward_equals_forward(ctx, width, depth):
    import torch
    from paper_2009_00705_amd import pmg
    net = pmg.Net(ctx, width=width, depth=depth, seed=11)
    th = net.get_params()[0]
    th[-1] = 0.25                                    # non-zero output bias
    net.set_params(th)
    # 10000 rows: two full chunks of 4096 and a ragged one; then 1500 rows: one partial chunk
    for n, seed in ((10000, 1), (1500, 2)):
        X = dev(_inputs(n, seed))
        y_ref = torch.empty(n, dtype=torch.float32, device="cuda")
        net.forward(X, y_ref)
        y = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(X, y)
        torch.cuda.synchronize()
        a, b = host(y), host(y_ref)
        assert np.isfinite(a).all(), (width, depth, n)
        assert np.array_equal(a, b), (width, depth, n, np.abs(a - b).max())
    net.close()


def test_noalloc_forward_rejects_wide_networks_and_accepts_empty_input(ctx):
    import torch
    from paper_2009_00705_amd import pmg
    wide = pmg.Net(ctx, width=257, depth=1, seed=3)
    X = dev(_inputs(64, 4))
    y = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(pmg.PmgError) as e:
        wide.forward_noalloc(X, y)
    assert e.value.code == -1 and "256" in str(e.value)
    assert float(y.abs().max()) == 0.0               # outputs untouched on rejection
    wide.close()
    net = pmg.Net(ctx, width=64, depth=2, seed=3)
    empty = torch.empty((0, 7), dtype=torch.float32, device="cuda")
    net.forward_noalloc(empty, torch.empty(0, dtype=torch.float32, device="cuda"))
    net.close()
