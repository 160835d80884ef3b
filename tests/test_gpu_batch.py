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


# --- batched adjoint ---------------------------------------------------------

def _grad_batch(seed):
    rng = np.random.default_rng(seed)
    specs = []
    kinds = [("box", dict(W=3)), ("gauss", dict(sigma_s=2.5)), ("box", dict(W=30)),   # W = 30: streamed adjoint
             ("gauss", dict(sigma_s=10.0)), ("gauss", dict(sigma_s=1.2)), ("box", dict(W=9)),
             ("gauss", dict(sigma_s=4.0))]
    for b, (kind, kw) in enumerate(kinds):
        H, Wd = int(rng.integers(20, 130)), int(rng.integers(20, 170))
        specs.append(dict(kernel=kind, sigma_r=float(rng.uniform(15, 60)), height=H, width=Wd, grad=True, **kw))
    return specs


def test_batch_backward_matches_per_image():
    torch, P = _mods()
    specs = _grad_batch(21)
    batch = P.Batch(specs)
    assert all(s >= 0 for s in batch.image_status)
    imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], 500 + i), dtype=torch.float32, device="cuda")
            for i, s in enumerate(specs)]
    for rep in range(2):
        gouts = [torch.tensor(synthimg.gen1(s["height"], s["width"], 600 + 10 * rep + i) / 255.0 - 0.5,
                              dtype=torch.float32, device="cuda") for i, s in enumerate(specs)]
        gins, gs = batch.backward(imgs, gouts)
        torch.cuda.synchronize()
        gs = gs.cpu().numpy()
        for i, s in enumerate(specs):
            kw = {k: v for k, v in s.items() if k not in ("kernel", "sigma_r", "height", "width")}
            plan = P.Plan(s["kernel"], s["sigma_r"], s["height"], s["width"], **kw)
            ref, rs = plan.backward(imgs[i], gouts[i])
            torch.cuda.synchronize()
            ref, rs = ref.cpu().numpy().astype(np.float64), rs.cpu().numpy()
            got = gins[i].cpu().numpy().astype(np.float64)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"rep {rep} image {i} {s['kernel']} W={plan.info.W} N={plan.info.N}: df rel {err:.2e} "
                  f"dsr {gs[i, 0]:.6e} vs {rs[0]:.6e} dss {gs[i, 1]:.6e} vs {rs[1]:.6e}", flush=True)
            assert err <= 1e-4, (rep, i)
            assert abs(gs[i, 0] - rs[0]) <= 1e-4 * abs(rs[0]), (rep, i)
            if s["kernel"] == "gauss":
                assert abs(gs[i, 1] - rs[1]) <= 1e-4 * abs(rs[1]), (rep, i)
            else:
                assert np.isnan(gs[i, 1])


def test_batch_backward_matches_autograd():
    from oracle import grad as GR
    torch, P = _mods()
    specs = [dict(kernel="gauss", sigma_s=2.0, sigma_r=30.0, height=40, width=52, grad=True),
             dict(kernel="box", W=4, sigma_r=25.0, height=33, width=45, grad=True),
             dict(kernel="gauss", sigma_s=9.0, sigma_r=40.0, height=50, width=61, grad=True)]  # W = 27
    batch = P.Batch(specs)
    imgs = [torch.tensor(synthimg.gen1(s["height"], s["width"], 700 + i), dtype=torch.float32, device="cuda")
            for i, s in enumerate(specs)]
    gouts = [torch.tensor(synthimg.gen2(s["height"], s["width"], 800 + i) / 255.0 - 0.5, dtype=torch.float32,
                          device="cuda") for i, s in enumerate(specs)]
    gins, gs = batch.backward(imgs, gouts)
    torch.cuda.synchronize()
    gs = gs.cpu().numpy()
    for i, s in enumerate(specs):
        kind = s["kernel"]
        W = s["W"] if kind == "box" else P.bf_order("gauss", 30.0, sigma_s=s["sigma_s"]).W
        df, dsr, dss = GR.vjp_autograd(imgs[i].cpu().numpy().astype(np.float64),
                                       gouts[i].cpu().numpy().astype(np.float64), kind, s.get("sigma_s"), W,
                                       s["sigma_r"], batch.N[i], 127.5)
        got = gins[i].cpu().numpy().astype(np.float64)
        assert np.abs(got - df).max() <= 1e-3 * np.abs(df).max(), i
        assert abs(gs[i, 0] - dsr) <= 1e-3 * abs(dsr), i
        if kind == "gauss":
            assert abs(gs[i, 1] - dss) <= 1e-3 * abs(dss), i


def test_wide_range_image_reported():
    # lambda above 170 runs only on the single-image wide-range path: the batch
    # reports that image as unsupported and keeps the others
    torch, P = _mods()
    from paper_1603_08109_amd import _lib as L
    batch = P.Batch([dict(kernel="gauss", sigma_s=2.0, sigma_r=30.0, height=40, width=50),
                     dict(kernel="gauss", sigma_s=2.0, sigma_r=6.0, height=40, width=50)])
    assert batch.image_status[0] >= 0 and batch.image_status[1] == L.BF_EUNSUPPORTED


def _own_plan(spec):
    # whether the batch's plain forward runs this image on its own plan's streamed passes
    import paper_1603_08109_amd as P
    from paper_1603_08109_amd import _lib as L
    kw = {k: v for k, v in spec.items() if k not in ("kernel", "sigma_r", "grad")}
    return P.bf_order(spec["kernel"], spec["sigma_r"], **kw).path == L.BF_PATH_STREAMED


def test_batch_saved_state_pair():
    # bf_batch_forward_saved / bf_batch_backward_saved: the same outputs as the
    # graphed forward (to rounding where the graphed forward takes the image's own
    # streamed plan and the saved form the fused tiles: both within the oracle
    # tolerance) and, from the same forward state (the same kernel writes it),
    # exactly the recomputing adjoint's gradients; the W = 30 box image takes the
    # streamed adjoint from the saved planes as well
    torch, P = _mods()
    specs = _grad_batch(33)
    tol = [1e-3 if _own_plan(s) else 1e-5 for s in specs]
    assert 1e-3 in tol and 1e-5 in tol
    batch = P.Batch(specs)
    assert all(s >= 0 for s in batch.image_status)
    imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], 900 + i), dtype=torch.float32, device="cuda")
            for i, s in enumerate(specs)]
    gouts = [torch.tensor(synthimg.gen1(s["height"], s["width"], 950 + i) / 255.0 - 0.5, dtype=torch.float32,
                          device="cuda") for i, s in enumerate(specs)]
    ref_out = [o.clone() for o in batch.forward(imgs)]
    ref_gin, ref_gs = batch.backward(imgs, gouts)
    ref_gin = [g.clone() for g in ref_gin]
    ref_gs = ref_gs.clone()
    saved = batch.new_saved()
    for rep in range(2):
        out = batch.forward(imgs, saved=saved)
        gin, gs = batch.backward(imgs, gouts, saved=saved)
        torch.cuda.synchronize()
        for i in range(len(specs)):
            assert torch.abs(out[i] - ref_out[i]).max().item() <= tol[i], (rep, i)
            assert torch.equal(gin[i], ref_gin[i]), (rep, i)
        assert torch.equal(torch.nan_to_num(gs, nan=7.0), torch.nan_to_num(ref_gs, nan=7.0)), rep


def test_batch_saved_state_errors():
    torch, P = _mods()
    plain = P.Batch([dict(kernel="gauss", sigma_s=2.0, sigma_r=30.0, height=20, width=30)])
    x = [torch.zeros(20, 30, device="cuda")]
    with pytest.raises(P.BFError):
        plain.forward(x, saved=plain.new_saved())                      # planned without BF_FLAG_GRAD
    g = P.Batch([dict(kernel="gauss", sigma_s=2.0, sigma_r=30.0, height=20, width=30, grad=True)])
    with pytest.raises(ValueError):
        g.forward(x, saved=[torch.empty(10, device="cuda")])           # too small


def test_side_streams_on_a_caller_stream():
    # images with Gaussian W >= 16 take their own streamed plans on the batch's side streams (more
    # of them than side streams), the others the persistent launch; three graph replays with new
    # inputs on a non-default caller stream, each image against the oracle, and the stream's order
    # kept: a kernel queued behind the call on the same stream sees the finished outputs
    torch, P = _mods()
    specs = [dict(kernel="gauss", sigma_s=ss, sigma_r=sr, height=H, width=Wd)
             for ss, sr, H, Wd in [(6.0, 30.0, 90, 130), (2.0, 25.0, 70, 64), (10.0, 40.0, 120, 75),
                                   (15.0, 30.0, 80, 200), (7.0, 20.0, 64, 64), (1.5, 50.0, 33, 170),
                                   (12.0, 35.0, 100, 100), (8.5, 45.0, 66, 140)]]
    batch = P.Batch(specs)
    assert all(s >= 0 for s in batch.image_status)
    stream = torch.cuda.Stream()
    for rep in range(3):
        imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], 700 + 10 * rep + i), dtype=torch.float32,
                             device="cuda") for i, s in enumerate(specs)]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            outs = batch.forward(imgs, stream=stream)
            sums = torch.stack([o.double().sum() for o in outs])  # queued behind the call on `stream`
        torch.cuda.synchronize()
        for i, s in enumerate(specs):
            W = K.support("gauss", sigma_s=s["sigma_s"])
            f32 = imgs[i].cpu().numpy().astype(np.float64)
            ref = _oracle(f32, s, batch.N[i], W)
            got = outs[i].cpu().numpy().astype(np.float64)
            assert np.abs(got - ref).max() <= TOL, (rep, i)
            assert abs(sums[i].item() - got.sum()) <= 1e-6 * abs(got.sum()), (rep, i)


def test_forward_is_one_graph_launch():
    # wide supports (Gaussian sigma_s = 25, box W = 75 on 2^20 pixels) next to narrow ones: the wide
    # images run their own streamed plans, and the whole forward (parameter copy, persistent tiles,
    # side-stream launches) replays as ONE graph launch per call with no other launch; the persistent
    # launch is planned for the narrow images only (its LDS is that of W = 9, not W = 75)
    torch, P = _mods()
    specs = [dict(kernel="gauss", sigma_s=25.0, sigma_r=30.0, height=300, width=280),
             dict(kernel="box", W=75, sigma_r=30.0, height=1024, width=1024),
             dict(kernel="gauss", sigma_s=2.0, sigma_r=25.0, height=90, width=130),
             dict(kernel="box", W=4, sigma_r=40.0, height=70, width=64),
             dict(kernel="gauss", sigma_s=3.0, sigma_r=30.0, height=64, width=200)]
    batch = P.Batch(specs)
    assert all(s >= 0 for s in batch.image_status)
    info = batch.get_info()
    assert info["images_streamed"] == 2 and info["images_persistent"] == 3
    # largest fused-tile LDS of a W <= 9 image (32-row tiles): region (32 + 18) x 83 floats plus
    # the row-pass buffer (32 + 18) x 65 floats
    assert 0 < info["persistent_lds_bytes"] <= 4 * (50 * 83 + 4 + 50 * 65)
    plans = []
    for s in specs:
        d = dict(s)
        plans.append(P.Plan(d.pop("kernel"), d.pop("sigma_r"), **d))
    stream = torch.cuda.Stream()
    for rep in range(3):
        imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], 900 + 10 * rep + i), dtype=torch.float32,
                             device="cuda") for i, s in enumerate(specs)]
        torch.cuda.synchronize()
        before = batch.get_info()
        with torch.cuda.stream(stream):
            outs = batch.forward(imgs, stream=stream)
        after = batch.get_info()
        assert after["forward_graph_launches"] == before["forward_graph_launches"] + 1
        assert after["forward_direct_launches"] == 0
        torch.cuda.synchronize()
        for i, s in enumerate(specs):
            ref = plans[i].forward(imgs[i])
            torch.cuda.synchronize()
            assert (outs[i] - ref).abs().max().item() <= 1e-4, (rep, i)
        if rep == 0:
            for i, s in enumerate(specs):
                f32 = imgs[i].cpu().numpy().astype(np.float64)
                got = outs[i].cpu().numpy().astype(np.float64)
                W = s["W"] if s["kernel"] == "box" else K.support("gauss", sigma_s=s["sigma_s"])
                px = synthimg.sample_pixels(s["height"], s["width"], 40, W, 20, 910 + i)
                w2 = K.taps2d(s["kernel"], s.get("sigma_s"), W if s["kernel"] == "box" else None)
                ref = G.gpa_pairwise_at(f32, px, w2, s["sigma_r"], batch.N[i], 127.5)
                assert np.abs(got[px[:, 0], px[:, 1]] - ref).max() <= TOL, i


def test_backward_is_one_graph_launch():
    # images on streamed plans of their own (Gaussian W = 30 and W = 18, box W = 40 on 2^20 pixels)
    # next to narrow ones, none on the shared streamed adjoint or with the reflecting border: every
    # adjoint call, recomputing or from saved state, with or without the sigma gradients, is ONE graph
    # launch (one capture per combination), and each replay, on other inputs and output gradients,
    # matches the per-image plans' adjoints
    torch, P = _mods()
    specs = [dict(kernel="gauss", sigma_s=10.0, sigma_r=30.0, height=150, width=170, grad=True),
             dict(kernel="gauss", sigma_s=6.0, sigma_r=25.0, height=120, width=90, grad=True),
             dict(kernel="box", W=40, sigma_r=40.0, height=1024, width=1024, grad=True),
             dict(kernel="gauss", sigma_s=2.0, sigma_r=35.0, height=80, width=100, grad=True),
             dict(kernel="box", W=3, sigma_r=20.0, height=60, width=70, grad=True)]
    batch = P.Batch(specs)
    assert all(s >= 0 for s in batch.image_status)
    info = batch.get_info()
    assert info["images_streamed"] == 3 and info["images_persistent"] == 2
    plans = []
    for s in specs:
        d = dict(s)
        plans.append(P.Plan(d.pop("kernel"), d.pop("sigma_r"), **d))
    stream = torch.cuda.Stream()
    saved = batch.new_saved()
    # (from saved state, sigma gradients asked)
    cases = [(False, True), (False, False), (True, True), (False, True), (True, False), (True, True)]
    for rep, (use_saved, want_sigma) in enumerate(cases):
        imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], 1200 + 10 * rep + i), dtype=torch.float32,
                             device="cuda") for i, s in enumerate(specs)]
        gouts = [torch.tensor(synthimg.gen1(s["height"], s["width"], 1300 + 10 * rep + i) / 255.0 - 0.5,
                              dtype=torch.float32, device="cuda") for i, s in enumerate(specs)]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            if use_saved:
                batch.forward(imgs, saved=saved, stream=stream)
            before = batch.get_info()
            gins, gs = batch.backward(imgs, gouts, want_sigma=want_sigma, saved=saved if use_saved else None,
                                      stream=stream)
            after = batch.get_info()
        assert after["backward_graph_launches"] == before["backward_graph_launches"] + 1, rep
        assert after["backward_direct_launches"] == 0, rep
        torch.cuda.synchronize()
        assert (gs is not None) == want_sigma
        g = gs.cpu().numpy() if want_sigma else None
        for i, s in enumerate(specs):
            ref, rs = plans[i].backward(imgs[i], gouts[i])
            torch.cuda.synchronize()
            ref, rs = ref.cpu().numpy().astype(np.float64), rs.cpu().numpy()
            got = gins[i].cpu().numpy().astype(np.float64)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"rep {rep} saved={use_saved} sigma={want_sigma} image {i} {s['kernel']} W={plans[i].info.W} "
                  f"N={plans[i].info.N}: df rel {err:.2e}", flush=True)
            assert err <= 1e-4, (rep, i)
            if want_sigma:
                assert abs(g[i, 0] - rs[0]) <= 1e-4 * abs(rs[0]), (rep, i)
                if s["kernel"] == "gauss":
                    assert abs(g[i, 1] - rs[1]) <= 1e-4 * abs(rs[1]), (rep, i)
                else:
                    assert np.isnan(g[i, 1]), (rep, i)
