"""GPU parity of the batched persistent forward (bf_batch_forward) against the
FP64 oracle and against per-image bf_forward launches, including hipGraph
replays with eager work in between."""
import numpy as np
import pytest

import synthimg
from oracle import gpa as G
from oracle import kernels as K

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _small_batch(seed):
    rng = np.random.default_rng(seed)
    specs = []
    for b in range(12):
        H, Wd = int(rng.integers(1, 160)), int(rng.integers(1, 200))
        if b % 3 == 0:
            specs.append(dict(kernel="box", W=int(rng.integers(0, 12)), sigma_r=float(rng.uniform(15, 60)),
                              height=H, width=Wd))
        else:
            specs.append(dict(kernel="gauss", sigma_s=float(rng.uniform(0.7, 6)),
                              sigma_r=float(rng.uniform(12, 60)), height=H, width=Wd))
    return specs


def _oracle(f32, spec, N, W):
    kind = spec["kernel"]
    w1 = K.taps1d(kind, spec.get("sigma_s"), W if kind == "box" else None)
    return G.gpa_alg2(f32, w1, spec["sigma_r"], N, 127.5)


def test_small_batch_matches_oracle_and_replays():
    torch, P = _mods()
    specs = _small_batch(3)
    batch = P.Batch(specs)
    assert all(s >= 0 for s in batch.image_status)
    for rep in range(3):
        imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], 100 * rep + i), dtype=torch.float32,
                             device="cuda") for i, s in enumerate(specs)]
        outs = batch.forward(imgs)
        # eager work between replays
        junk = torch.randn(1000, 1000, device="cuda").sum()
        torch.cuda.synchronize()
        for i, s in enumerate(specs):
            f32 = imgs[i].cpu().numpy().astype(np.float64)
            W = s.get("W") if s["kernel"] == "box" else P.bf_order("gauss", 30.0, sigma_s=s["sigma_s"]).W
            ref = _oracle(f32, s, batch.N[i], W)
            err = np.abs(outs[i].cpu().numpy().astype(np.float64) - ref).max()
            assert err <= TOL, (rep, i, s, err)
        del junk


def test_batch_equals_per_image_plans():
    torch, P = _mods()
    specs = _small_batch(5)
    batch = P.Batch(specs)
    imgs = [torch.tensor(synthimg.gen1(s["height"], s["width"], i), dtype=torch.float32, device="cuda")
            for i, s in enumerate(specs)]
    outs = batch.forward(imgs)
    for i, s in enumerate(specs):
        d = dict(s)
        plan = P.Plan(d.pop("kernel"), d.pop("sigma_r"), **d)
        ref = plan.forward(imgs[i])
        torch.cuda.synchronize()
        assert plan.info.N == batch.N[i]
        assert (outs[i] - ref).abs().max().item() <= 1e-4


def test_tune_keeps_results():
    torch, P = _mods()
    specs = _small_batch(9)
    batch = P.Batch(specs)
    imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], i), dtype=torch.float32, device="cuda")
            for i, s in enumerate(specs)]
    outs0 = [o.clone() for o in batch.forward(imgs)]
    outs = [torch.empty_like(x) for x in imgs]
    chosen = batch.tune(imgs, outs)
    assert chosen >= 0
    outs1 = batch.forward(imgs)
    torch.cuda.synchronize()
    for a, b in zip(outs0, outs1):
        assert (a - b).abs().max().item() <= 1e-4


def test_workload4_batch():
    # 256 images, sizes U{64..1024} x U{64..768}, sigma_s ~ U[2,15], sigma_r ~ U[10,60]
    torch, P = _mods()
    specs = synthimg.batch_params(256, 4000)
    per = [dict(kernel="gauss", sigma_s=s["sigma_s"], sigma_r=s["sigma_r"], height=s["height"],
                width=s["width"]) for s in specs]
    batch = P.Batch(per)
    assert all(st >= 0 for st in batch.image_status)
    imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], s["seed"]), dtype=torch.float32,
                         device="cuda") for s in specs]
    outs = batch.forward(imgs)
    torch.cuda.synchronize()
    worst = 0.0
    for i in range(0, 256, 37):  # sampled images, sampled pixels
        s = specs[i]
        f32 = imgs[i].cpu().numpy().astype(np.float64)
        W = P.bf_order("gauss", s["sigma_r"], sigma_s=s["sigma_s"]).W
        px = synthimg.sample_pixels(s["height"], s["width"], 150, W, 50, 4000 + i)
        w2 = K.taps2d("gauss", s["sigma_s"])
        ref = G.gpa_pairwise_at(f32, px, w2, s["sigma_r"], batch.N[i], 127.5)
        got = outs[i].cpu().numpy().astype(np.float64)[px[:, 0], px[:, 1]]
        worst = max(worst, np.abs(got - ref).max())
    print(f"workload-4 sampled max err {worst:.3e}", flush=True)
    assert worst <= TOL
