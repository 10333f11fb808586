"""Allocation-free inference of the temperature-step network: the forward
pass of pa_mlp_forward_noalloc (device pointers, fixed per-device scratch)
equals pa_mlp_forward's output bit for bit, on consecutive calls whose batch
shrinks, and a batch beyond the scratch limit is refused before any launch."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pa():
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU")
    from paper_2006_00561_amd import binding
    binding.lib()
    import torch
    assert torch.cuda.is_available(), "torch sees no GPU beside the library"
    torch.cuda.set_device(0)
    return binding


@pytest.mark.parametrize("n_in,width,depth,batches",
                         [(8, 64, 3, (1500, 37, 1)), (5, 100, 2, (700, 300))])
def test_noalloc_forward_equals_forward(pa, n_in, width, depth, batches):
    import torch
    rng = np.random.default_rng(n_in * 1000 + width)
    stream = torch.cuda.current_stream().cuda_stream
    mlp = pa.MLP(n_in, width, depth, seed=11, stream=stream)
    mlp.set_norm(rng.normal(0, 0.5, n_in), rng.uniform(0.5, 2.0, n_in),
                 -4.5, 1.3)
    for B in batches:
        X = rng.normal(0, 1.5, (B, n_in)).astype(np.float32)
        y_ref = mlp.forward(X)
        Xd = torch.from_numpy(X).to("cuda")
        yd = torch.full((B,), float("nan"), dtype=torch.float32,
                        device="cuda")
        torch.cuda.synchronize()
        print("noalloc forward n_in=%d width=%d depth=%d B=%d"
              % (n_in, width, depth, B), flush=True)
        mlp.forward_noalloc(Xd.data_ptr(), B, yd.data_ptr())
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        assert np.array_equal(y.view(np.uint32), y_ref.view(np.uint32))
    mlp.close()


def test_noalloc_refuses_batch_beyond_scratch(pa):
    import torch
    mlp = pa.MLP(8, 64, 3, seed=2)
    limit = 262144 // 64          # PA_MLP_NOALLOC_MAX_ELEMS / max(width, n_in)
    Xd = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    yd = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(pa.PAError):
        mlp.forward_noalloc(Xd.data_ptr(), limit + 1, yd.data_ptr())
    with pytest.raises(pa.PAError):
        mlp.forward_noalloc(Xd.data_ptr(), 0, yd.data_ptr())
    mlp.close()
