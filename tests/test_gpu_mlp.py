"""The MLP kernels against the FP64 oracle on the same bfloat16 weights (GPU),
training progress, and what the trained network gains over the plain sweep."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from paper_2607_18991_amd import learned, nz

pytestmark = pytest.mark.gpu


def device_params(seed):
    p32 = (np.random.default_rng(seed).normal(0, 0.25, size=nz.NZ_MLP_NPARAM)).astype(np.float32)
    bits = learned.to_bf16_bits(p32)
    return p32, bits, omlp.bf16_to_f64(bits)


def rows(B, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.integers(0, 2, size=(B, 7)), rng.normal(size=(B, 1))], axis=1)
    return x.astype(np.float32)


@pytest.mark.parametrize("B", [1, 7, 33, 135])
def test_forward_backward_match_oracle(B):
    _, bits, p64 = device_params(B)
    x = rows(B, B + 1)
    dy = np.random.default_rng(B + 2).normal(size=(B, 2)).astype(np.float32)
    pb = torch.from_numpy(bits.view(np.int16)).cuda()
    xd = torch.from_numpy(x).cuda()
    y = torch.empty((B, 2), dtype=torch.float32, device="cuda")
    act = torch.empty((B, nz.NZ_MLP_NACT), dtype=torch.float32, device="cuda")
    g = torch.empty(nz.NZ_MLP_NPARAM, dtype=torch.float32, device="cuda")
    nz.nz_mlp_forward(pb, xd, y, act)
    nz.nz_mlp_backward(pb, xd, act, torch.from_numpy(dy).cuda(), g)
    torch.cuda.synchronize()
    y_o, cache = omlp.forward(p64, x.astype(np.float64))
    g_o = omlp.backward(p64, x.astype(np.float64), cache, dy.astype(np.float64))
    assert np.allclose(y.cpu().numpy(), y_o, rtol=1e-5, atol=1e-5)
    scale = np.abs(g_o).max()
    err = np.abs(g.cpu().numpy() - g_o)
    assert (err <= 1e-4 * np.maximum(np.abs(g_o), 1e-2 * scale)).all(), err.max()


def test_loss_matches_oracle():
    B = 50
    rng = np.random.default_rng(3)
    y = rng.normal(size=(B, 2)).astype(np.float32)
    t = rng.normal(size=(B, 2)).astype(np.float32)
    w = rng.uniform(0.5, 4, size=B).astype(np.float32)
    dy = torch.empty((B, 2), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    nz.nz_mlp_loss(torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(w).cuda(), dy, loss)
    lo, dyo = omlp.loss_and_dy(y, t, w)
    assert float(loss.item()) == pytest.approx(lo, rel=1e-5)
    assert np.allclose(dy.cpu().numpy(), dyo, rtol=1e-5, atol=1e-7)


def test_adam_matches_oracle_and_rounds_bf16_exactly():
    p32, bits, _ = device_params(9)
    rng = np.random.default_rng(10)
    g = rng.normal(size=nz.NZ_MLP_NPARAM).astype(np.float32)
    w = torch.from_numpy(p32.copy()).cuda()
    wb = torch.from_numpy(bits.view(np.int16).copy()).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    gd = torch.from_numpy(g).cuda()
    wo, mo, vo = p32.astype(np.float64), np.zeros(nz.NZ_MLP_NPARAM), np.zeros(nz.NZ_MLP_NPARAM)
    for step in range(1, 4):
        nz.nz_mlp_adam(w, wb, gd, m, v, [1e-3, 0.9, 0.999, 1e-8, 1e-4], step)
        wo, mo, vo = omlp.adam_step(wo, mo, vo, g.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, 1e-4, step)
    torch.cuda.synchronize()
    w_gpu = w.cpu().numpy()
    assert np.allclose(w_gpu, wo, rtol=1e-6, atol=1e-7)
    assert (wb.cpu().numpy().view(np.uint16) == omlp.bf16_round(w_gpu)).all()


def test_training_reduces_loss_on_smooth_targets():
    pts = []
    for L in (4, 6, 8, 12, 16):
        for m in range(1, 128, 3):
            z = nz.nz_coordination(m)
            mean = 1.55 / (z + 1.0) * (1 + 1.0 / L)
            std = mean * 0.5 * L**-1.5
            pts.append(dict(L=L, mask=m, count=100, mean=mean, std=std, ln_mean=np.log(mean), ln_std=np.log(std)))
    model = learned.train(pts, steps=600, lr=3e-3, log_every=100)
    hist = model.meta["loss_history"]
    assert hist[-1][1] < 0.05 * hist[0][1]


def test_learned_prefill_gain_over_plain():
    """Train on small lattices, predict a larger one, and compare the learned
    prefill with the plain sweep: identical n* and mass, several times fewer
    sequential steps."""
    from gpu_util import run_batch

    masks = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F, 0x12, 0x44]
    train_jobs = [dict(L=L, zone_mask=m, seed=777 + L, nsamples=400) for L in (6, 8, 10) for m in masks]
    ns, _, _, _ = run_batch(train_jobs)
    pts, off = [], 0
    for j in train_jobs:
        pts.append(learned.aggregate(j["L"], j["zone_mask"], ns[off:off + j["nsamples"]]))
        off += j["nsamples"]
    model = learned.train(pts, steps=1500, lr=3e-3)
    test = [dict(L=12, zone_mask=m, seed=4321, nsamples=200) for m in masks]
    plain = learned.plan_band_only(model, test)
    pn, pm, _, pst = run_batch(plain)
    lj = model.plan(test)
    ln, lm, _, lst = run_batch(lj)
    assert (pn == ln).all() and (pm == lm).all()
    assert pst["serial_steps"] >= 3 * lst["serial_steps"], (pst, lst)
    assert lst["backoffs"] <= 0.05 * sum(j["nsamples"] for j in test)
