"""Training and evaluation driver of the learned troubled-cell indicator.

Orchestration only: every feature, label, forward, backward and Adam step
runs in the library's kernels (dg_mlp_*).  The driver
  1. runs the plain limited scheme on several seeded blast-wave states and
     records (features, plain-detector label) pairs of the projected initial
     state and of every pre-limiter stage (all positives, a fraction of
     negatives),
  2. trains the network on the device,
  3. measures the false-negative rate (cells the network would skip while
     the plain detector fires) on held-out seeds and picks the gate mlp_lo.
"""
import numpy as np

from .binding import DG, DG_LIM_CHAR, DG_LIM_LEARNED, DG_LIM_POS, DG_LIM_TVB


def record_dataset(gpu, fields, steps, cap, q_pos=1.0, q_neg=0.05, seed=0, sigma=None):
    """Run the plain limited scheme from each field and record samples.
    Returns (X, y, nrows, sigma)."""
    import torch
    X = torch.zeros((cap, 256), dtype=torch.int16, device="cuda")
    y = torch.zeros(cap, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    w = gpu.empty_state()
    for i, f in enumerate(fields):
        gpu.project_field(f, w)
        if sigma is None:
            sigma = gpu.mlp_scale(w)
            gpu.mlp_set(None, sigma, seed=seed)
        # the initial limiting of the projected state is recorded too
        gpu.mlp_record(X, y, cnt, q_pos=q_pos, q_neg=q_neg, seed=seed + 7919 * i)
        gpu.limit(w)
        gpu.step(w, steps)
        gpu.mlp_record(None)
    torch.cuda.synchronize()
    n = min(int(cnt.item()), cap)
    return X, y, n, sigma


def false_negative_rate(gpu, X, y, n, lo):
    """Fraction of plain-detector positives the gate (p < lo) would skip, and
    the fraction of all recorded cells it skips."""
    import torch
    prob = torch.zeros(max(n, 1), device="cuda")
    gpu.mlp_forward(X, n, prob)
    torch.cuda.synchronize()
    p = prob[:n].cpu().numpy()
    lab = y[:n].cpu().numpy() > 0.5
    fn = float(((p < lo) & lab).sum() / max(lab.sum(), 1))
    skip = float((p < lo).mean())
    return fn, skip, p, lab


def choose_lo(p, lab, target_fn=0.0, margin=0.5):
    """Gate threshold: the target_fn quantile of the probabilities of the
    plain detector's positives (target_fn = 0: the smallest), times a safety
    margin, at most 0.5.  A skipped troubled cell is never limited
    in that stage and its oscillation feeds the next stages, so the default
    admits no false negative on the validation set."""
    pos = np.sort(p[lab])
    if pos.size == 0:
        return 0.5
    k = int(np.floor(target_fn * pos.size))
    q = pos[k] if k < pos.size else pos[-1]
    return float(min(margin * q, 0.5))


def train_indicator(workloads, n=128, d=3, train_seeds=range(4001, 4033), val_seeds=range(4101, 4103), steps=4,
                    cap=12 << 20, q_pos=0.1, q_neg=0.006, epochs=4, batch=4096, lr=2e-3, precision=1, stream=None,
                    seed=1):
    """Train on blast states of the given seeds; returns a dict with the
    parameters, feature scales, losses and validation statistics.  The
    defaults record about 11M labelled cells from 32 blast seeds (13
    pre-limiter states each: the projection and 4 steps x 3 stages)."""
    lim = DG_LIM_TVB | DG_LIM_CHAR | DG_LIM_POS
    gpu = DG(3, d, n, limiter=lim, precision=precision, stream=stream)
    Xt, yt, nt, sigma = record_dataset(gpu, [workloads.Blast(s) for s in train_seeds], steps, cap, q_pos=q_pos,
                                       q_neg=q_neg, seed=seed)
    losses = gpu.mlp_train(Xt, yt, nt, batch=batch, epochs=epochs, lr=lr, seed=seed) if nt >= batch else []
    params = gpu.mlp_get()
    pos_frac = float(yt[:nt].mean().item()) if nt else 0.0
    del Xt, yt
    Xv, yv, nv, _ = record_dataset(gpu, [workloads.Blast(s) for s in val_seeds], steps, cap // 2, q_pos=q_pos,
                                   q_neg=q_neg, seed=seed + 1, sigma=sigma)
    # the second recording re-installed nothing: restore the trained network
    gpu.mlp_set(params, sigma)
    _, _, p, lab = false_negative_rate(gpu, Xv, yv, nv, 0.0)
    lo = choose_lo(p, lab)
    fn, skip, _, _ = false_negative_rate(gpu, Xv, yv, nv, lo)
    out = dict(params=params, sigma=sigma, losses=[float(x) for x in losses], n_train=nt,
               pos_frac_train=pos_frac, n_val=nv, lo=lo, val_fn_rate=fn, val_skip_frac=skip,
               n_train_seeds=len(train_seeds))
    gpu.close()
    return out
