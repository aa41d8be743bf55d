"""DTW as a training loss: gradient descent of a barycentre of warped, noisy
copies of a template through DTWFunction (forward and backward in the HIP
kernels), checked against the FP64 oracle's DTW of the trained barycentre.
The distances of Section 2 and their path gradient are the only part of the
loop this library computes; the optimizer is the caller's."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import check_gpu_paths, close

pytestmark = pytest.mark.gpu


def test_dtw_loss_barycentre_training():
    g = gen.rng(4700)
    L, P, w = 64, 256, 7
    template = gen.standardise(gen.random_walk(L, g))
    S = gen.as_f32(np.stack([gen.standardise(gen.warped_copy(template, g)) for _ in range(P)]))
    St = torch.from_numpy(S).cuda()

    def loss_of(b):
        return eap.DTWFunction.apply(b.unsqueeze(0).expand(P, L).contiguous(), St, w).mean()

    B = torch.nn.Parameter(St.mean(0).clone())  # the Euclidean mean: blurred by the warps
    opt = torch.optim.Adam([B], lr=0.05)
    losses = []
    for _ in range(150):
        opt.zero_grad()
        loss = loss_of(B)
        loss.backward()
        assert torch.isfinite(B.grad).all()
        opt.step()
        losses.append(loss.item())
    final = loss_of(B.detach()).item()
    assert final < 0.7 * losses[0], (losses[0], final)
    assert min(losses[-10:]) <= min(losses[:10])
    # better than any of 16 of the copies used as the barycentre (a medoid)
    with torch.no_grad():
        medoid = min(eap.DTWFunction.apply(St[i].unsqueeze(0).expand(P, L).contiguous(), St, w)
                     .mean().item() for i in range(16))
    assert final < medoid, (final, medoid)
    # the trained barycentre's loss is the oracle's
    b = gen.as_oracle(B.detach().cpu().numpy())
    ref = float(np.mean([oracle.dtw(b, gen.as_oracle(S[p]), w) for p in range(P)]))
    assert close(final, ref), (final, ref)
    # the per-pair gradients at the trained barycentre, on the GPU's own
    # paths (a trained barycentre sits near many path ties, where float32
    # rounding picks one of several optimal paths)
    Bx = B.detach().unsqueeze(0).expand(P, L).contiguous().requires_grad_(True)
    d = eap.DTWFunction.apply(Bx, St, w)
    d.mean().backward()
    gx = Bx.grad.cpu().numpy()
    dp, rr, cr = eap.dtw_path(Bx.detach(), St, w)
    check_gpu_paths(Bx.detach().cpu().numpy(), S, w, d.detach().cpu().numpy(), rr.cpu().numpy(),
                    cr.cpu().numpy(), gx, None, np.full(P, 1.0 / P), grad_abs=1e-5 / P)
