"""Surrogate speed-up at fixed error: data from batched DD bursts, ensemble
training, a spread threshold calibrated on held-out states, and the cost of
DD and of the surrogate at equal error.

Every device computation goes through the library's calls (dd_burst_batch,
dd_mlp_train_step, dd_surrogate_rates); numpy does the bookkeeping.

States and errors.  A *state* fixes what the surrogate sees (applied stress;
per loop its slip system, radius and mobility: hence the per-system resolved
shear stresses and mobile/sessile line densities, the 36 features); its
*microstructures* (loop centres, phases, Burgers signs) are drawn from a
second seed (workloads.burst_instance_state).  One burst of 200 glide steps
gives the 12 burst-averaged slip rates of one microstructure.  The reference
of a held-out state s is the mean Rbar_s over its M microstructures.  Errors
over a set K of states are relative root-sum-square errors,
    E(pred) = ( sum_K |pred_s - Rbar_s|^2 / sum_K |Rbar_s|^2  -  E1^2 / M )^(1/2),
with the reference's own noise E1^2 / M removed in quadrature; E1 (one burst
against its state's mean) comes from the per-state sample covariances.  DD
reaches an error e with n(e) = ceil(E1^2 / e^2) bursts per state, at the
measured mean burst time each.

Fallback.  The ensemble spread (dd_surrogate_rates) flags points for DD.  The
threshold for a target error e is calibrated on half of the held-out states
(the largest threshold whose kept states have error <= e) and applied to the
other half, on which the kept fraction and error are reported.  A flagged
state costs n(e) bursts; the surrogate's cost per state is its inference time
per point plus the fallback fraction times that.

Noise floor.  With targets of relative noise E1 (single bursts), the
network's error falls no faster than N^(-1/2) in the number of training
bursts N while the variance term dominates; the learning curve (N/4, N/2, N)
is fitted by that law and by a free power law and extrapolated to the N that
would reach 5 %.
"""
from __future__ import annotations

import math
import time

import numpy as np

STATE_BASE_TRAIN, MICRO_BASE_TRAIN = 2_000_000, 5_000_000
STATE_BASE_HELD, MICRO_BASE_HELD = 3_000_000, 4_000_000
BATCH = 512
N_STEPS = 200


def _dev():
    import torch
    return torch.device("cuda:0")


def burst_data(states, seeds, state_base, micro_base, log=None, n_steps=N_STEPS):
    """One mixed-precision burst of n_steps glide steps per (state,
    microstructure): features X [states][seeds][36] and rates Y
    [states][seeds][12] (float64), the seconds spent in the burst calls and
    the number of bursts."""
    import torch

    import paper_2005_02498_amd as dd
    from paper_2005_02498_amd import workloads as W

    dev = _dev()
    mat = {"mu": W.MU, "nu": W.NU, "a": W.CORE_A, "B": W.DRAG_B}
    pairs = [(s, k) for s in range(states) for k in range(seeds)]
    X, Y, sec = [], [], 0.0
    for b0 in range(0, len(pairs), BATCH):
        ins = [W.burst_instance_state(state_base + s, micro_base + seeds * s + k) for s, k in pairs[b0:b0 + BATCH]]
        bt = W.pack(ins)
        d = dict(x=torch.tensor(bt.x, device=dev), sn=torch.tensor(bt.seg_nodes, device=dev),
                 b=torch.tensor(bt.burgers, device=dev), n=torch.tensor(bt.normal, device=dev),
                 p=torch.tensor(bt.pinned, device=dev), s=torch.tensor(bt.sigma_app, device=dev),
                 v=torch.tensor(bt.volume, device=dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, f = dd.dd_burst_batch(bt.node_off, bt.seg_off, d["x"], d["sn"], d["b"], d["n"], d["p"], d["s"], d["v"],
                                 mat, 2, dd.DD_MIXED, 20.0, n_steps, W.DT, want_features=True)
        torch.cuda.synchronize()
        sec += time.perf_counter() - t0
        X.append(f.cpu().numpy())
        Y.append(r.cpu().numpy())
        if log:
            log(f"bursts {min(b0 + BATCH, len(pairs))}/{len(pairs)}")
    X = np.concatenate(X).reshape(states, seeds, 36)
    Y = np.concatenate(Y).reshape(states, seeds, 12)
    return X, Y, sec, len(pairs)


def noise_vs_length(states, seeds, lengths, log=None):
    """The single-burst scatter E1 against the burst length: the same
    held-out states and microstructures, run for each number of glide steps
    in `lengths`.  A scatter that comes from the finite time average falls
    as the bursts get longer; one that comes from the microstructures (the
    spread of the time averages of different microstructures of one state)
    does not."""
    rows = []
    for n in lengths:
        _, Y, sec, nb = burst_data(states, seeds, STATE_BASE_HELD, MICRO_BASE_HELD, log, n_steps=n)
        Rbar = Y.mean(1)
        _, E1 = state_errors(Rbar, Y)
        rel = np.sqrt(Y.var(1, ddof=1).sum(1)) / np.maximum(np.linalg.norm(Rbar, axis=1), 1e-300)
        rows.append({"steps": n, "error_single_burst": E1, "median_state_scatter": float(np.median(rel)),
                     "mean_state_rate_norm": float(np.mean(np.linalg.norm(Rbar, axis=1))),
                     "bursts": nb, "seconds": sec})
        if log:
            log(f"{n} steps: E1 = {E1:.3f}")
    return {"study": "single-burst scatter against burst length", "states": states,
            "microstructures_per_state": seeds, "rows": rows}


def train(X, Y, epochs, members=4, seed=12345, log=None):
    """An ensemble trained on features X [n][36] and targets Y [n][12] with
    the library's training step (Adam, batches of 1024, learning rate 1e-3,
    then 3e-4 and 1e-4 over the last 40 % of the epochs); 10 % of the rows
    are a validation split, and the parameters with the lowest validation
    loss (checked every 5 epochs) are kept.  Returns (model, info)."""
    import torch

    import paper_2005_02498_amd as dd
    from paper_2005_02498_amd import workloads as W

    dev = _dev()
    dens_scale, dens_floor = 1.0 / W.B_SI ** 2, 1e10
    Xt = X.copy()
    Xt[:, 12:] = np.log10(np.maximum(Xt[:, 12:], 0) * dens_scale + dens_floor)
    in_shift = Xt.mean(0)
    in_scale = 1.0 / np.maximum(Xt.std(0), 1e-6)
    out_shift = Y.mean(0)
    out_scale = np.maximum(Y.std(0), 1e-30)
    model = dd.SurrogateModel(members, seed)
    model.set_log_densities(dens_scale, dens_floor)
    model.set_scaling(in_shift, in_scale, out_shift, out_scale)
    rng = np.random.default_rng(0)
    order = rng.permutation(len(X))
    n_val = max(1, len(X) // 10)
    val, trn = order[:n_val], order[n_val:]
    Xd = torch.tensor(X[trn], dtype=torch.float32, device=dev)
    Yd = torch.tensor(Y[trn], dtype=torch.float32, device=dev)
    Xv = torch.tensor(X[val], dtype=torch.float32, device=dev)
    Yv = Y[val]
    nb = 1024
    steps = max(1, len(trn) // nb)
    best, best_ep, best_params = float("inf"), -1, None
    t0 = time.perf_counter()
    for ep in range(epochs):
        lr = 1e-3 if ep < 0.6 * epochs else (3e-4 if ep < 0.85 * epochs else 1e-4)
        perm = torch.tensor(rng.permutation(len(trn)), device=dev)
        for k in range(steps):
            idx = perm[k * nb:(k + 1) * nb]
            dd.dd_mlp_train_step(model, Xd[idx].contiguous(), Yd[idx].contiguous(), lr)
        if ep % 5 == 4 or ep == epochs - 1:
            pv, _, _ = dd.dd_surrogate_rates(model, Xv, 0.05)
            vloss = float(np.mean(((pv.cpu().numpy() - Yv) / out_scale) ** 2))
            if vloss < best:
                best, best_ep = vloss, ep
                best_params = [model.get_params(m) for m in range(members)]
    for m in range(members):
        model.set_params(m, best_params[m])
    torch.cuda.synchronize()
    info = {"rows": int(len(X)), "epochs": epochs, "best_epoch": best_ep, "validation_loss": best,
            "seconds": time.perf_counter() - t0}
    if log:
        log(f"trained on {len(X)} rows: best epoch {best_ep}, validation loss {best:.4f}")
    # the spread floor (rate units): 10 % of the training RMS rate
    model.set_spread_floor(0.1 * float(np.sqrt(np.mean(Y ** 2))))
    return model, info


def predict(model, X):
    """Rates [n][12] and ensemble spread [n] for features X [n][36]."""
    import torch

    import paper_2005_02498_amd as dd
    pr, sp, _ = dd.dd_surrogate_rates(model, torch.tensor(X, dtype=torch.float32, device=_dev()), 0.05)
    return pr.cpu().numpy().astype(np.float64), sp.cpu().numpy().astype(np.float64)


def state_errors(pred, Yho, keep=None):
    """(E, E1) over the kept held-out states: E the noise-corrected error of
    pred [S][12] against the M-microstructure means of Yho [S][M][12], E1 the
    single-burst error over the same states."""
    if keep is None:
        keep = np.ones(len(Yho), bool)
    Y = Yho[keep]
    M = Y.shape[1]
    Rbar = Y.mean(1)
    den = float(np.sum(Rbar ** 2))
    if den == 0.0:
        return 0.0, 0.0
    E1sq = float(np.sum(Y.var(1, ddof=1)) / den)
    raw = float(np.sum((pred[keep] - Rbar) ** 2) / den)
    return math.sqrt(max(raw - E1sq / M, 0.0)), math.sqrt(E1sq)


def calibrate(spread, pred, Yho, e):
    """The largest spread threshold whose kept states (spread <= threshold)
    have error <= e; -1 when no non-empty kept set reaches e."""
    best = -1.0
    for t in np.unique(spread):
        keep = spread <= t
        if state_errors(pred, Yho, keep)[0] <= e:
            best = float(t)
    return best


def inference_seconds_per_point(model, X):
    """Inference time per point of one 1,048,576-point call (points drawn from X)."""
    import torch

    import paper_2005_02498_amd as dd
    n = 1 << 20
    rng = np.random.default_rng(1)
    F = torch.tensor(X[rng.integers(0, len(X), n)], dtype=torch.float32, device=_dev())
    for _ in range(2):
        dd.dd_surrogate_rates(model, F, 0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        dd.dd_surrogate_rates(model, F, 0.05)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps / n


def speedups(model, Xho, Yho, t_burst, t_inf, targets):
    """Held-out evaluation: calibration on the even states, report on the odd
    ones, for each target error e (None: the surrogate's own error on the
    odd states)."""
    pred, spread = predict(model, Xho[:, 0])
    cal, ev = np.arange(len(Xho)) % 2 == 0, np.arange(len(Xho)) % 2 == 1
    E_all, E1 = state_errors(pred, Yho)
    E_ev, _ = state_errors(pred[ev], Yho[ev])
    out = {"error_surrogate": E_all, "error_surrogate_evaluation_half": E_ev, "error_single_burst": E1,
           "spread_median": float(np.median(spread)),
           "fallback_fraction_at_fixed_tol": {str(t): float((spread > t).mean()) for t in (0.05, 0.1, 0.2, 0.5)}}
    # spread vs error: the states in four spread quartiles
    q = np.quantile(spread, [0.25, 0.5, 0.75])
    bins = np.digitize(spread, q)
    out["error_by_spread_quartile"] = [state_errors(pred, Yho, bins == b)[0] for b in range(4)]
    rows = {}
    for e in targets:
        name = "at_surrogate_error" if e is None else f"at_{e:g}"
        e = E_ev if e is None else e
        thr = calibrate(spread[cal], pred[cal], Yho[cal], e)
        keep = spread[ev] <= thr if thr >= 0 else np.zeros(int(ev.sum()), bool)
        fb = 1.0 - float(keep.mean())
        e_keep = state_errors(pred[ev], Yho[ev], keep)[0] if keep.any() else None
        n = max(1, math.ceil((E1 / e) ** 2))
        dd_cost = n * t_burst
        sur_cost = t_inf + fb * dd_cost
        rows[name] = {"error": e, "spread_threshold": thr, "fallback_fraction": fb,
                      "error_kept_states": e_keep, "dd_bursts_per_state": n, "dd_seconds_per_state": dd_cost,
                      "surrogate_seconds_per_state": sur_cost, "speedup": dd_cost / sur_cost,
                      "speedup_without_fallback": dd_cost / t_inf}
    out.update(rows)
    return out


def fit_learning_curve(pts, t_burst, e=0.05):
    """Fits of the held-out error against the number of training bursts N,
    extrapolated to the N that reaches e: the variance law E^2 = c / N (least
    squares in E^2) and a power law E = A N^-p (least squares in log E)."""
    N = np.array([p["training_bursts"] for p in pts], float)
    E = np.array([p["error"] for p in pts])
    c = float(np.sum(E ** 2 / N) / np.sum(1.0 / N ** 2))
    slope, icpt = np.polyfit(np.log(N), np.log(E), 1)
    p_exp = -float(slope)
    n_pow = float(math.exp((math.log(e) - icpt) / slope)) if slope < 0 else float("inf")
    return {"points": pts,
            "variance_law": {"fit": "E^2 = c / N", "c": c, "bursts_for_5_percent": c / e ** 2,
                             "hours_of_bursts": c / e ** 2 * t_burst / 3600.0},
            "power_law": {"fit": "E = A N^-p", "A": float(math.exp(icpt)), "p": p_exp,
                          "bursts_for_5_percent": n_pow, "hours_of_bursts": n_pow * t_burst / 3600.0}}


def study(train_states, train_seeds, held_states, held_seeds, epochs, learning_curve=True, log=None):
    """The full study; returns a JSON-ready dict."""
    t_start = time.perf_counter()
    Xtr, Ytr, sec_tr, nb_tr = burst_data(train_states, train_seeds, STATE_BASE_TRAIN, MICRO_BASE_TRAIN, log)
    Xho, Yho, sec_ho, nb_ho = burst_data(held_states, held_seeds, STATE_BASE_HELD, MICRO_BASE_HELD, log)
    t_burst = (sec_tr + sec_ho) / (nb_tr + nb_ho)
    res = {"study": "surrogate speed-up at fixed error",
           "burst": f"{N_STEPS} glide steps, mixed precision, 2 Gauss points, batches of {BATCH}",
           "training_states": train_states, "training_microstructures_per_state": train_seeds,
           "heldout_states": held_states, "heldout_microstructures_per_state": held_seeds,
           "mean_burst_seconds": t_burst, "data_generation_seconds": sec_tr + sec_ho}
    # (a) one row per burst: every microstructure's rates as a target
    model, info = train(Xtr.reshape(-1, 36), Ytr.reshape(-1, 12), epochs, log=log)
    t_inf = inference_seconds_per_point(model, Xho[:, 0])
    res["inference_seconds_per_point"] = t_inf
    res["per_burst_targets"] = {"train": info, **speedups(model, Xho, Yho, t_burst, t_inf, (None, 0.1, 0.05))}
    model.close()
    # (b) one row per state: the mean over its microstructures (the same bursts)
    if train_seeds > 1:
        model, info = train(Xtr[:, 0], Ytr.mean(1), epochs, log=log)
        res["per_state_mean_targets"] = {"train": info,
                                         **speedups(model, Xho, Yho, t_burst, t_inf, (None, 0.1, 0.05))}
        model.close()
    # learning curve of (a): the noise floor
    if learning_curve:
        pts = []
        for frac in (0.25, 0.5, 1.0):
            ns = max(1, int(train_states * frac))
            if frac == 1.0:
                e = res["per_burst_targets"]["error_surrogate"]
            else:
                m, _ = train(Xtr[:ns].reshape(-1, 36), Ytr[:ns].reshape(-1, 12), epochs, log=log)
                e = state_errors(predict(m, Xho[:, 0])[0], Yho)[0]
                m.close()
            pts.append({"training_bursts": ns * train_seeds, "error": e})
        res["learning_curve"] = fit_learning_curve(pts, t_burst)
    res["total_seconds"] = time.perf_counter() - t_start
    return res
