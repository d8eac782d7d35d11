"""Allocation-free inference entry point (gsis_mlp_forward_noalloc) against the allocating one
(gsis_mlp_forward): the same kernels over the same rows, so the outputs must agree bit for bit, on two calls in
a row (the second smaller), for BF16 and FP32 weights, with a batch larger than one scratch chunk."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rows(n, n_in, seed):
    return np.random.default_rng(seed).standard_normal((n, n_in)).astype(np.float32)


@pytest.mark.parametrize("bf16", [True, False], ids=["bf16", "fp32"])
def test_noalloc_forward_matches_forward(bf16):
    import torch

    from paper_2601_03935_amd.warmstart import MLP

    stream = torch.cuda.current_stream()
    width, n_in, n_out = 256, 7, 7
    m = MLP(n_in=n_in, width=width, n_out=n_out, bf16=bf16, seed=11, stream=stream.cuda_stream)
    # 8 MiB of scratch holds 4,096 rows at width 256: the first call goes through three chunks, the second one
    for n, seed in ((10000, 5), (1500, 6)):
        x = _rows(n, n_in, seed)
        ref = m.forward(x)
        xd = torch.from_numpy(x).to("cuda:0")
        yd = torch.full((n, n_out), float("nan"), dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        m.forward_noalloc(xd.data_ptr(), yd.data_ptr(), n)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        assert np.isfinite(y).all()
        np.testing.assert_array_equal(y, ref)
    m.close()


def test_noalloc_forward_argument_errors():
    from paper_2601_03935_amd.gsis import GsisError
    from paper_2601_03935_amd.warmstart import MLP

    m = MLP(width=64, bf16=True, seed=1)
    with pytest.raises(GsisError, match="row count"):
        m.forward_noalloc(0, 0, -1)
    with pytest.raises(GsisError, match="null input"):
        m.forward_noalloc(0, 0, 4)
    m.forward_noalloc(0, 0, 0)  # an empty batch launches nothing
    m.close()
