"""GPU parity of the learned troubled-cell indicator: BF16-MFMA forward and
backward against the oracle network (BF16-rounding mode) on fixed batches,
features and plain-detector labels against the oracle, the fused gate of
the limiter against features + forward, and a training run that learns."""
import numpy as np
import pytest

import workloads as wl
from oracle import dg, limiters, mlp
from parity_util import make_pair, to_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pub(P):
    return np.concatenate([p.ravel() for p in P]).astype(np.float32)


def _unpub(v):
    out, q = [], 0
    for fin, fout in mlp.LAYERS:
        out.append(v[q:q + fin * fout].reshape(fin, fout).astype(np.float64)); q += fin * fout
        out.append(v[q:q + fout].astype(np.float64)); q += fout
    return out


def _bf16_tensor(x):
    """float64 numpy -> device bf16 bits (int16 tensor) with the oracle's rounding."""
    r = mlp.bf16_round(x).astype(np.float32)
    bits = (r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.as_tensor(bits, device="cuda").contiguous()


def _gpu_handle(limiter=0, n=6, d=3):
    from paper_1806_02343_amd import DG
    return DG(3, d, n, limiter=limiter, mlp_lo=0.2, mlp_hi=0.6)


def test_forward_and_gradients_match_oracle():
    print("case mlp grad", flush=True)
    rng = np.random.default_rng(1)
    P = mlp.init_params(2)
    P = [p + (0.05 * rng.normal(size=p.shape) if p.ndim == 1 else 0) for p in P]  # nonzero biases
    X = rng.normal(size=(64, 256))
    y = (rng.uniform(size=64) > 0.6).astype(np.float64)
    gpu = _gpu_handle()
    gpu.mlp_set(_pub(P), np.ones(9))
    Xd = _bf16_tensor(X)
    yd = torch.as_tensor(y.astype(np.float32), device="cuda")
    loss_g, G = gpu.mlp_grad(Xd, yd, 64)
    Pq = _unpub(_pub(P))  # the parameters as the GPU holds them (FP32)
    loss_o, Go = mlp.backward(Pq, X, y, bf16=True)
    assert abs(loss_g - loss_o) <= 1e-3 * loss_o
    Gg = _unpub(G)
    for a, b in zip(Gg, Go):
        assert np.abs(a - b).max() <= 2e-2 * np.abs(b).max() + 1e-7
    prob = torch.zeros(64, device="cuda")
    gpu.mlp_forward(Xd, 64, prob)
    torch.cuda.synchronize()
    po, _ = mlp.forward(Pq, X, bf16=True)
    assert np.abs(prob.cpu().numpy() - po).max() < 5e-3
    # against the FP64 network (no BF16 rounding anywhere): the BF16 operands
    # (8 significant bits) leave a few per cent per element, ~1e-2 of each
    # layer's largest gradient
    loss_64, G64 = mlp.backward(Pq, X, y, bf16=False)
    assert abs(loss_g - loss_64) <= 1e-2 * loss_64
    rel = [np.abs(a - b).max() / np.abs(b).max() for a, b in zip(Gg, G64)]
    print("gradient error vs the FP64 network, per parameter block:", ["%.1e" % r for r in rel], flush=True)
    assert max(rel) < 1e-2, rel                       # measured <= 4.1e-3
    p64, _ = mlp.forward(Pq, X, bf16=False)
    assert np.abs(prob.cpu().numpy() - p64).max() < 2e-2


def test_adam_steps_match_oracle():
    """Three Adam steps on one full batch (dg_mlp_train with batch = rows)
    against the oracle's BF16-rounding gradients and adam_update: the update
    of an element is lr times a ratio of moments that the gradients' BF16
    noise moves by a few per cent, so the parameters agree to a small
    fraction of lr (and within the 3 lr an element can move at all)."""
    print("case mlp adam", flush=True)
    rng = np.random.default_rng(4)
    P = mlp.init_params(6)
    B, lr, k = 256, 1e-3, 3
    X = rng.normal(size=(B, 256))
    y = (rng.uniform(size=B) > 0.5).astype(np.float64)
    gpu = _gpu_handle()
    gpu.mlp_set(_pub(P), np.ones(9))
    Pq = _unpub(_pub(P))
    Xq = mlp.bf16_round(X)
    gpu.mlp_train(_bf16_tensor(X), torch.as_tensor(y.astype(np.float32), device="cuda"), B, batch=B, epochs=k, lr=lr,
                  seed=3)
    Pg = _unpub(gpu.mlp_get())
    Po = [p.copy() for p in Pq]
    M = [np.zeros_like(p) for p in Po]
    V = [np.zeros_like(p) for p in Po]
    for t in range(1, k + 1):
        _, G = mlp.backward([mlp.bf16_round(p) if p.ndim == 2 else p for p in Po], Xq, y, bf16=True)
        mlp.adam_update(Po, G, M, V, t, lr)
    d = np.concatenate([np.abs(a - b).ravel() for a, b in zip(Pg, Po)])
    moved = np.concatenate([np.abs(a - b).ravel() for a, b in zip(Po, Pq)])
    assert np.median(moved) > 0.5 * lr                      # the steps did move the parameters
    assert np.median(d) < 0.02 * lr and d.max() < 2 * k * lr, (np.median(d) / lr, d.max() / lr)


def _blast_state(n=6, d=3):
    gpu, wg, orc, wo = make_pair(3, d, n, dg.GLM, field=wl.Blast(2000), limiter=7)
    return gpu, wg, orc, wo


def test_features_and_labels_match_oracle():
    print("case mlp features", flush=True)
    from paper_1806_02343_amd import DG
    for d in (2, 3):
        gpu0, wg, orc, wo = _blast_state(d=d)
        sigma = mlp.feature_scale(orc, wo)
        sg = gpu0.mlp_scale(wg)
        assert np.allclose(sg, sigma, rtol=1e-12)
        gpu0.mlp_set(None, None, seed=3)
        X = torch.zeros((orc.mesh.ncells, 256), dtype=torch.int16, device="cuda")
        gpu0.mlp_features(wg, X)
        torch.cuda.synchronize()
        Xg = (X.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        Xo = mlp.bf16_round(mlp.features(orc, wo, sigma))
        # equal up to one bf16 ulp; entries that are zero in exact arithmetic
        # carry projection rounding noise (~1e-17) on both sides
        assert np.all(np.abs(Xg - Xo) <= 2 ** -7 * np.abs(Xo) + 1e-12)
        y = torch.zeros(orc.mesh.ncells, device="cuda")
        gpu0.mlp_labels(wg, y)
        torch.cuda.synchronize()
        ch = orc.timestep(wo)[1]
        _, tr = limiters.slope_limit(orc, wo, ch=ch)
        assert np.array_equal(y.cpu().numpy() > 0.5, tr)


def test_gate_counts_match_features_and_forward():
    print("case mlp gate", flush=True)
    from paper_1806_02343_amd import DG, DG_LIM_CHAR, DG_LIM_LEARNED, DG_LIM_POS, DG_LIM_TVB
    lim = DG_LIM_TVB | DG_LIM_CHAR | DG_LIM_POS | DG_LIM_LEARNED
    gpu, wg, orc, wo = make_pair(3, 3, 6, dg.GLM, field=wl.Blast(2000), limiter=lim, mlp_lo=0.45, mlp_hi=0.55)
    sigma = mlp.feature_scale(orc, wo)
    gpu.mlp_set(None, sigma, seed=5)
    C = orc.mesh.ncells
    X = torch.zeros((C, 256), dtype=torch.int16, device="cuda")
    gpu.mlp_features(wg, X)
    prob = torch.zeros(C, device="cuda")
    gpu.mlp_forward(X, C, prob)
    torch.cuda.synchronize()
    p = prob.cpu().numpy()
    st = gpu.limit(wg, stats=True)
    assert st["n_mlp_flagged"] == int((p >= 0.55).sum())
    assert st["n_fallback"] == int(((p >= 0.45) & (p < 0.55)).sum())


def test_gated_limit_matches_oracle():
    """The learned gate inside dg_limit (Sec. 4.2 detect-then-limit with the
    network in front): cells whose probability (oracle features, oracle
    forward with the GPU's parameters) is below mlp_lo skip the detector and
    stay bitwise; every other cell is limited as the oracle limits it.  Cells
    whose probability lies within 1e-2 of mlp_lo (the BF16 forward's spread)
    are left out of the comparison."""
    print("case mlp gated limit", flush=True)
    from paper_1806_02343_amd import DG, DG_LIM_CHAR, DG_LIM_LEARNED, DG_LIM_POS, DG_LIM_TVB
    gpu0, wg0, orc, wo = make_pair(3, 3, 6, dg.GLM, field=wl.Blast(2000), limiter=7)
    sigma = mlp.feature_scale(orc, wo)
    gpu0.mlp_set(None, sigma, seed=5)
    Pq = _unpub(gpu0.mlp_get())
    # spread the logits so that the probabilities cover (0, 1)
    Pq[6] = Pq[6] * 40.0
    p, _ = mlp.forward(Pq, mlp.bf16_round(mlp.features(orc, wo, sigma)), bf16=True)
    lo = float(np.quantile(p, 0.5))
    lim = DG_LIM_TVB | DG_LIM_CHAR | DG_LIM_POS | DG_LIM_LEARNED
    gpu = DG(3, 3, 6, limiter=lim, mlp_lo=lo, mlp_hi=1.5)
    gpu.mlp_set(_pub(Pq), sigma)
    wg = torch.as_tensor(orc.to_abi(wo, gpu.ld), device="cuda")
    st = gpu.limit(wg, stats=True)
    wgc = to_cells(wg, orc.mesh.ncells)
    skip = p < lo
    sure = np.abs(p - lo) > 1e-2
    ch = orc.timestep(wo)[1]
    wl_, tr = limiters.slope_limit(orc, wo, ch=ch)
    wl_[skip] = wo[skip]
    wo2, _ = limiters.positivity(orc, wl_)
    assert skip[sure].any() and (~skip[sure]).any() and (tr & ~skip & sure).any()
    ref_trig = int((tr & ~skip)[sure].sum())
    gpu_trig_bound = st["n_tvb_triggered"]
    assert abs(gpu_trig_bound - ref_trig) <= int((~sure).sum())
    err = np.abs(wgc[sure] - wo2[sure]).max(axis=1) / np.abs(wo2).max()
    assert np.all(err < 1e-12), err.max()


def test_training_learns_a_separable_rule():
    print("case mlp train", flush=True)
    rng = np.random.default_rng(7)
    n = 8192
    X = rng.normal(size=(n, 256)) * 0.5
    y = (X[:, 3] + 0.5 * X[:, 100] - 0.3 * X[:, 200] > 0.2).astype(np.float32)
    gpu = _gpu_handle()
    gpu.mlp_set(None, np.ones(9), seed=11)
    Xd = _bf16_tensor(X)
    yd = torch.as_tensor(y, device="cuda")
    losses = gpu.mlp_train(Xd, yd, n, batch=512, epochs=8, lr=3e-3, seed=1)
    assert losses[-1] < 0.5 * losses[0], losses
    prob = torch.zeros(n, device="cuda")
    gpu.mlp_forward(Xd, n, prob)
    torch.cuda.synchronize()
    acc = ((prob.cpu().numpy() > 0.5) == (y > 0.5)).mean()
    assert acc > 0.9, acc
    # parameters round-trip through the host
    P = gpu.mlp_get()
    gpu.mlp_set(P, np.ones(9))
    prob2 = torch.zeros(n, device="cuda")
    gpu.mlp_forward(Xd, n, prob2)
    torch.cuda.synchronize()
    assert torch.equal(prob, prob2)


def test_recording_inside_steps():
    print("case mlp record", flush=True)
    gpu, wg, orc, wo = _blast_state(n=6, d=3)
    gpu.mlp_scale(wg)
    gpu.mlp_set(None, None, seed=1)
    gpu.limit(wg)
    cap = 4096
    X = torch.zeros((cap, 256), dtype=torch.int16, device="cuda")
    y = torch.full((cap,), -1.0, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    # every cell of every stage: 6 stages x 216 cells
    gpu.mlp_record(X, y, cnt, q_pos=1.0, q_neg=1.0, seed=3)
    gpu.step(wg, 2)
    gpu.mlp_record(None)
    torch.cuda.synchronize()
    k = int(cnt.item())
    assert k == 6 * 216
    assert torch.all((y[:k] == 0.0) | (y[:k] == 1.0))
    assert torch.all(y[k:] == -1.0)
    # the recorded features are those of real cells (first feature = rho mean / s_rho > 0)
    f0 = (X[:k, 0].to(torch.int32) & 0xFFFF).cpu().numpy().astype(np.uint32) << 16
    assert np.all(f0.view(np.float32) > 0)


def test_training_driver_on_blast_states():
    """The driver records plain-detector labels inside limited steps, trains,
    and picks a gate with no false negative on the held-out seeds; a run with
    the gate limits no cell the plain detector would leave alone and differs
    from the plain run only through the cells it skips."""
    print("case mlp driver", flush=True)
    from paper_1806_02343_amd import DG, DG_LIM_CHAR, DG_LIM_LEARNED, DG_LIM_POS, DG_LIM_TVB
    from paper_1806_02343_amd.learned import train_indicator
    info = train_indicator(wl, n=24, d=3, train_seeds=range(4001, 4004), val_seeds=range(4029, 4030), steps=4,
                           cap=1 << 16, q_neg=0.2, epochs=6, batch=512, lr=3e-3, precision=1)
    assert info["n_train"] > 4 * 512
    assert 0.0 < info["pos_frac_train"] < 1.0
    assert info["losses"][-1] < info["losses"][0], info["losses"]
    assert 0.0 <= info["lo"] <= 0.5
    assert info["val_fn_rate"] == 0.0
    lim = DG_LIM_TVB | DG_LIM_CHAR | DG_LIM_POS
    plain = DG(3, 3, 24, limiter=lim, precision=1)
    gated = DG(3, 3, 24, limiter=lim | DG_LIM_LEARNED, precision=1, mlp_lo=info["lo"], mlp_hi=0.5)
    gated.mlp_set(info["params"], info["sigma"])
    wp, wq = plain.empty_state(), gated.empty_state()
    plain.project_field(wl.Blast(2000), wp)
    gated.project_field(wl.Blast(2000), wq)
    sp = plain.limit(wp, stats=True)
    sq = gated.limit(wq, stats=True)
    # the gate only removes cells from the plain detector's work: cells below
    # the gate are skipped, every other cell runs the plain detector
    skipped = plain.ncells - sq["n_fallback"] - sq["n_mlp_flagged"]
    assert 0 <= skipped <= plain.ncells
    assert sq["n_tvb_triggered"] <= sp["n_tvb_triggered"]
    assert sp["n_tvb_triggered"] - sq["n_tvb_triggered"] <= skipped
    if skipped == 0:
        assert sq["n_tvb_triggered"] == sp["n_tvb_triggered"]
        assert torch.equal(wp, wq)
