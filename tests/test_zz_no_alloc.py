"""mlp_grad_noalloc (the library's per-GPU scratch, no caller workspace) against mlp_grad (a
caller workspace): the same kernels and partition, so the gradients and losses agree bit for bit,
over two calls in a row, the second with fewer samples than the first."""
import numpy as np
import pytest

from paper_1312_2234_amd import lbm

DEV = "cuda:0"


def _net(rng):
    th = np.concatenate([rng.normal(0, 0.3, 1024), rng.normal(0, 0.05, 64), rng.normal(0, 0.15, 4096),
                         rng.normal(0, 0.05, 64), rng.normal(0, 0.1, 1024), rng.normal(0, 0.05, 16)])
    norm = np.concatenate([rng.normal(0, 0.1, 16), rng.uniform(0.5, 2.0, 16), rng.uniform(0.2, 1.0, 16)])
    return th.astype(np.float32), norm.astype(np.float32)


@pytest.mark.gpu
def test_mlp_grad_noalloc_matches_mlp_grad():
    import torch

    rng = np.random.default_rng(31)
    th, norm = _net(rng)
    P = lbm.mlp_pack(torch.from_numpy(th).to(DEV), torch.from_numpy(norm).to(DEV))
    # 70,001 samples: more 64-sample chunks than workgroups (the grid strides); then 3,001
    for B in (70001, 3001):
        raw = torch.from_numpy(rng.normal(0, 1, (B, 16)).astype(np.float32)).to(DEV)
        tgt = torch.from_numpy(rng.normal(0, 0.5, (B, 16)).astype(np.float32)).to(DEV)
        g_ref, l_ref = lbm.mlp_grad(P, raw, tgt)
        g, l = lbm.mlp_grad_noalloc(P, raw, tgt)
        torch.cuda.synchronize()
        print("B=%d loss %.6e / %.6e, max|grad| %.3e" % (B, float(l[0]), float(l_ref[0]),
                                                         float(g_ref.abs().max())))
        assert torch.isfinite(g_ref).all() and float(g_ref.abs().max()) > 0.0
        assert torch.equal(g, g_ref), "gradients differ"
        assert torch.equal(l, l_ref), "losses differ"


@pytest.mark.gpu
def test_mlp_grad_noalloc_rejects_bad_arguments():
    import torch

    rng = np.random.default_rng(32)
    th, norm = _net(rng)
    P = lbm.mlp_pack(torch.from_numpy(th).to(DEV), torch.from_numpy(norm).to(DEV))
    raw = torch.zeros((0, 16), dtype=torch.float32, device=DEV)
    with pytest.raises(RuntimeError):
        lbm.mlp_grad_noalloc(P, raw, raw)     # B = 0
