"""The no-allocation loss/gradient entry point (mce_model_loss_grad_noalloc)
against the allocating one (mce_model_loss_grad) through the C ABI: the same
kernels in the same order, so gradient and loss must be identical, also on a
second call with a smaller input that finds the first call's values in the
shared scratch array."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    import torch

    from paper_2212_01473_amd import learned

    rng = np.random.default_rng(seed)
    feat = np.stack([rng.uniform(0, 8, n), rng.uniform(0, 6, n), rng.uniform(0, 12, n), rng.uniform(0, 1, n)],
                    axis=1).astype(np.float32)
    target = rng.uniform(0, 10, n).astype(np.float32)
    model = learned.init_model(seed)
    # normalisation as fitted from the features, so the hidden units mix signs
    model[-8:-4] = feat.mean(axis=0)
    model[-4:] = feat.std(axis=0) + 1e-3
    return (torch.from_numpy(model).cuda(), torch.from_numpy(feat).cuda(), torch.from_numpy(target).cuda())


def test_noalloc_loss_grad_matches_allocating_entry_point(gpu_lib):
    import torch

    # the largest size first, then a smaller one (ragged against the 4096-sample
    # gradient chunks and the 256-sample blocks)
    for n, seed in ((gpu_lib.MCE_NOALLOC_MAX_SAMPLES, 1), (3001, 2)):
        model, feat, target = _inputs(n, seed)
        ref_grad, ref_loss = gpu_lib.model_loss_grad(model, feat, target)
        grad = torch.full((gpu_lib.MODEL_FLOATS,), float("nan"), dtype=torch.float32, device="cuda")
        loss = gpu_lib.model_loss_grad_noalloc(model, feat, target, grad)
        torch.cuda.synchronize()
        assert torch.equal(grad, ref_grad), n
        assert loss == ref_loss, n
        assert torch.all(grad[-8:] == 0)  # mean/std are not trained


def test_noalloc_rejects_sizes_beyond_its_limit(gpu_lib):
    import torch

    model, feat, target = _inputs(gpu_lib.MCE_NOALLOC_MAX_SAMPLES + 1, 3)
    grad = torch.zeros(gpu_lib.MODEL_FLOATS, dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.MCEError) as e:
        gpu_lib.model_loss_grad_noalloc(model, feat, target, grad)
    assert e.value.status == gpu_lib.MCE_ERR_INVALID_ARG
    assert "MCE_NOALLOC_MAX_SAMPLES" in str(e.value)
    with pytest.raises(gpu_lib.MCEError) as e:
        gpu_lib.model_loss_grad_noalloc(model, feat[:0], target[:0], grad)
    assert e.value.status == gpu_lib.MCE_ERR_INVALID_ARG
