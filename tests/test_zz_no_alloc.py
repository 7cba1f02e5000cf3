"""The allocation-free inference forward (semx_mlp_forward_noalloc) against
the existing forward (semx_mlp_forward) through the C ABI: same network,
same input, same GEMM kernels, so the outputs must agree to the last bits of
the FP32 SiLU; two calls in a row, the second with a smaller batch, plus the
size limit of the static workspace, and the FP64 reference as a sanity bound.

Also runs the first call of the process on a fresh network (the workspace
address is resolved once per device when a network is created)."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu

WIDTHS = [64, 512, 512, 512, 24576]   # the surrogate's network (64 -> 3 x 512 -> 16 x 512 x 3)


def _outputs(net, x, batch):
    import torch
    import paper_2606_12850_amd as P
    y_ref = torch.full((batch, WIDTHS[-1]), float("nan"), device="cuda")
    y_na = torch.full((batch, WIDTHS[-1]), float("nan"), device="cuda")
    P.semx_mlp_forward(net, x, batch, y_ref)
    P.semx_mlp_forward_noalloc(net, x, batch, y_na)
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


def test_noalloc_forward_matches_forward_twice():
    import torch
    import paper_2606_12850_amd as P
    rng = np.random.default_rng(7)
    theta = (M.he_uniform(WIDTHS, 5) + 0.01 * rng.standard_normal(M.num_params(WIDTHS))).astype(np.float32)
    net = P.semx_mlp_create(WIDTHS, 1024)
    P.semx_mlp_set_params(net, theta)
    for batch in (1024, 300):   # second call smaller: the workspace keeps the first call's data
        x = torch.from_numpy(rng.standard_normal((batch, WIDTHS[0])).astype(np.float32)).cuda()
        y_ref, y_na = _outputs(net, x, batch)
        assert np.all(np.isfinite(y_na))
        diff = float(np.max(np.abs(y_na - y_ref)) / np.max(np.abs(y_ref)))
        y64, _ = M.forward(theta.astype(np.float64), WIDTHS, x.cpu().numpy().astype(np.float64))
        e64 = rel_l2(y_na, y64)
        print(f"batch {batch}: max |noalloc - forward| / max |y| = {diff:.3e}; vs FP64 rel L2 {e64:.2e}")
        assert diff <= 1e-6
        assert e64 <= 2e-2   # the BF16 forward's bar against the FP64 reference
    P.semx_mlp_destroy(net)


def test_noalloc_forward_batch_limit():
    import torch
    import paper_2606_12850_amd as P
    net = P.semx_mlp_create([64, 512, 8], 16)
    P.semx_mlp_set_params(net, M.he_uniform([64, 512, 8], 1).astype(np.float32))
    # batch x widest hidden layer must stay within 2^21 floats: 4096 x 512 fits, 4097 does not
    x = torch.zeros((4097, 64), device="cuda")
    y = torch.zeros((4097, 8), device="cuda")
    P.semx_mlp_forward_noalloc(net, x, 4096, y)   # above the network's max_batch, within the workspace
    torch.cuda.synchronize()
    assert torch.all(torch.isfinite(y[:4096]))
    with pytest.raises(P.SemxError) as ei:
        P.semx_mlp_forward_noalloc(net, x, 4097, y)
    assert ei.value.code == P.SEMX_EINVAL
    with pytest.raises(P.SemxError) as ei:
        P.semx_mlp_forward_noalloc(net, x, 0, y)
    assert ei.value.code == P.SEMX_EINVAL
    P.semx_mlp_destroy(net)
