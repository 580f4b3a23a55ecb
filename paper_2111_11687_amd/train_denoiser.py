"""Training data, training, evaluation and the Monte Carlo-judged fallback of
the dose denoiser (denoiser.py).  Every dose map comes from the engine of
this package; every network step runs in the HIP library.

Training data: synthetic patients (phantoms.patient_phantom), each run
twice -- a low-history input with seed s + 10^6 and a high-history target
with seed s + 2*10^6 -- and cut into boxes at seeded positions inside the
body.

Fallback (organ_dose_with_fallback): the low-history run is made as two
independent halves A and B (the same phantom registered under two ids, so
their random streams differ).  Each half is denoised; the organ estimate is
the mean X_o of the two denoised organ means, with the estimated error

    e_o = sqrt(delta_o^2 + b_o^2),  delta_o = |X_o^A - X_o^B| / (2 X_o),

where b_o is the organ's calibrated bias (a high percentile of the held-out
organ errors).  Plain Monte Carlo judges the estimate: an organ is accepted
only if e_o <= tol and |X_o - M_o| <= 3 sigma_o, with M_o the Monte Carlo
organ mean of both halves and sigma_o its standard error (the organ mean is
unbiased).  Rejected organs fall back to Monte Carlo, continued on both
halves until 2 sigma_o / M_o <= tol; their Monte Carlo value is reported.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np

from . import binding as B
from . import denoiser as DN
from . import phantoms as P

PID_A, PID_B = 62, 63  # phantom ids used by these helpers


def _organ_sigma(sig_a, sig_b, m_a, m_b):
    """Standard error of the mean of two independent half estimates."""
    return 0.5 * np.sqrt((sig_a * m_a) ** 2 + (sig_b * m_b) ** 2)


def _run_map(eng, pid, n, seed):
    eng.run(pid, n, seed)
    rate, _ = eng.dose(pid)
    return rate


def pick_box(label, box_shape, rng, organ_fraction=0.0, n_organs=None):
    """A box of box_shape (d, h, w) clamped inside the volume.  With
    probability organ_fraction it is centred on a random voxel of a random
    organ (labels 1 .. n_organs - 1, the last label being the body
    remainder), else on a random point of the body's bounding box."""
    shape = label.shape
    if any(b > s for b, s in zip(box_shape, shape)):
        raise ValueError("box larger than the phantom")
    centre = None
    if organ_fraction > 0 and n_organs and rng.random() < organ_fraction:
        o = int(rng.integers(1, n_organs))
        vox = np.argwhere(label == o)
        if len(vox):
            centre = vox[int(rng.integers(len(vox)))]
    if centre is None:
        body = np.argwhere(label > 0)
        lo, hi = body.min(0), body.max(0)
        centre = [rng.integers(lo[a], hi[a] + 1) for a in range(3)]
    out = [int(np.clip(centre[a] - box_shape[a] // 2, 0, shape[a] - box_shape[a]))
           for a in range(3)]
    return tuple(out) + tuple(box_shape)


def make_samples(eng, seeds, n_lo, n_hi, box_shape, boxes_per_phantom, rng,
                 shape=(320, 256, 256), voxel_mm=(2.0, 2.0, 3.0), log=print,
                 organ_fraction=0.0):
    """(x0, target) device tensors of `boxes_per_phantom` boxes of each
    phantom of `seeds`.  The next phantom is generated on a host thread while
    the GPU runs the current one."""
    from concurrent.futures import ThreadPoolExecutor
    t = eng.torch
    dev = eng.device
    samples = []
    seeds = [int(s) for s in seeds]
    gen = lambda s: P.patient_phantom(shape=shape, voxel_mm=voxel_mm, seed=s)  # noqa: E731
    with ThreadPoolExecutor(1) as pool:
        nxt = pool.submit(gen, seeds[0]) if seeds else None
        for k, s in enumerate(seeds):
            t0 = time.perf_counter()
            prob = nxt.result()
            if k + 1 < len(seeds):
                nxt = pool.submit(gen, seeds[k + 1])
            t1 = time.perf_counter()
            eng.set_problem(PID_A, prob)
            lo = _run_map(eng, PID_A, n_lo, s + 10 ** 6)
            B.nmd_reset_tallies(eng.ctx, PID_A)
            hi = _run_map(eng, PID_A, n_hi, s + 2 * 10 ** 6)
            inp = eng.inputs[PID_A]
            for _ in range(boxes_per_phantom):
                box = pick_box(prob.label, box_shape, rng, organ_fraction, prob.n_organs)
                x0 = t.empty(tuple(box_shape) + (DN.IN_CH,), dtype=t.bfloat16, device=dev)
                tgt = t.empty(tuple(box_shape), dtype=t.float32, device=dev)
                scale = t.empty(2, dtype=t.float64, device=dev)
                B.nmd_nn_prepare(eng.ctx, prob.shape, box, lo, hi, inp["density"],
                                 inp["activity"], inp["label"], x0, tgt, scale)
                samples.append((x0, tgt))
            eng.sync()
            log("phantom %d: waited %.1f s for the host generator, Monte Carlo %.1f s" % (
                s, t1 - t0, time.perf_counter() - t1))
    return samples


def train(eng, net, samples, steps, lr=1e-3, seed=0, log_every=100, log=print,
          weight_floor=0.0):
    """Adam on randomly drawn samples with a cosine learning-rate decay;
    returns the logged (step, loss) pairs."""
    rng = np.random.default_rng(seed)
    shape = tuple(samples[0][1].shape)
    ws = DN.Workspace(eng, shape)
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        x0, tgt = samples[int(rng.integers(len(samples)))]
        ws.x0, ws.target = x0, tgt
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / steps))
        net.train_step(ws, max(lr_t, lr * 0.02), weight_floor=weight_floor)
        if it % log_every == 0 or it == steps - 1:
            loss = ws.loss_value(net)
            hist.append((it, loss))
            log("step %5d  loss %.5g  %.1f s" % (it, loss, time.perf_counter() - t0))
    return hist


def denoise_map(eng, net, pid, prob, dose_map, ws=None):
    """Denoised dose-rate map (FP64, Gy/s) of a whole phantom."""
    t = eng.torch
    if ws is None:
        ws = DN.Workspace(eng, prob.shape, train=False)
    inp = eng.inputs[pid]
    ws.prepare(eng, prob.shape, (0, 0, 0) + tuple(prob.shape), dose_map, inp["density"],
               inp["activity"], inp["label"])
    out = t.empty(prob.shape, dtype=t.float64, device=eng.device)
    net.predict(ws, out)
    return out


def _voxel_errors(x, ref, label):
    """Mean |relative error| and RMS relative error over body voxels whose
    reference dose exceeds 10% of the body mean."""
    body = label > 0
    thr = 0.1 * ref[body].mean()
    m = body & (ref > thr)
    rel = (x[m] - ref[m]) / ref[m]
    return float(np.abs(rel).mean()), float(np.sqrt((rel ** 2).mean()))


def evaluate(eng, net, seeds, n_lo, n_hi, shape=(320, 256, 256), voxel_mm=(2.0, 2.0, 3.0),
             log=print):
    """Voxel and organ errors of the low-history Monte Carlo and of its
    denoised version against the high-history Monte Carlo."""
    rows = []
    ws = None
    for s in seeds:
        prob = P.patient_phantom(shape=shape, voxel_mm=voxel_mm, seed=int(s))
        eng.set_problem(PID_A, prob)
        lo = _run_map(eng, PID_A, n_lo, int(s) + 10 ** 6)
        org_lo, _, sig_lo = eng.organs(PID_A)
        if ws is None or ws.shape != tuple(prob.shape):
            ws = DN.Workspace(eng, prob.shape, train=False)
        dn = denoise_map(eng, net, PID_A, prob, lo, ws)
        org_dn = B.nmd_organ_mean_map(eng.ctx, PID_A, dn, prob.n_organs)
        B.nmd_reset_tallies(eng.ctx, PID_A)
        hi = _run_map(eng, PID_A, n_hi, int(s) + 2 * 10 ** 6)
        org_hi, _, sig_hi = eng.organs(PID_A)
        lo_h, dn_h, hi_h = lo.cpu().numpy(), dn.cpu().numpy(), hi.cpu().numpy()
        lab = prob.label
        v_lo = _voxel_errors(lo_h, hi_h, lab)
        v_dn = _voxel_errors(dn_h, hi_h, lab)
        present = org_hi > 0  # organs with voxels at this voxel size
        den = np.where(present, org_hi, 1.0)
        e_lo = np.where(present, np.abs(org_lo - org_hi) / den, 0.0)
        e_dn = np.where(present, np.abs(org_dn - org_hi) / den, 0.0)
        rows.append({"seed": int(s), "voxel_lo": v_lo, "voxel_dn": v_dn,
                     "organ_lo": e_lo.tolist(), "organ_dn": e_dn.tolist(),
                     "sigma_lo": sig_lo.tolist(), "sigma_hi": sig_hi.tolist()})
        log("seed %d: voxel |rel| lo %.4f dn %.4f; organ max lo %.4f dn %.4f" % (
            s, v_lo[0], v_dn[0], e_lo.max(), e_dn.max()))
    return rows


def bias_table(rows, q=95.0):
    """Per-organ bias b_o: the q-th percentile of the denoised organ errors
    over the evaluation phantoms."""
    e = np.array([r["organ_dn"] for r in rows])
    return np.percentile(e, q, axis=0)


def plain_mc_to_tolerance(eng, prob, n_first, seed, tol=0.01, chunk=10 ** 8, max_decays=10 ** 10):
    """Plain Monte Carlo continued until 2 sigma_o / M_o <= tol for every
    organ.  Returns (organ means, relative sigmas, decays, seconds, reached)."""
    eng.set_problem(PID_A, prob)
    eng.sync()
    t0 = time.perf_counter()
    eng.run(PID_A, n_first, seed)
    n = n_first
    while True:
        org, _, sig = eng.organs(PID_A)
        worst = float(np.max(2 * sig))
        if worst <= tol or n >= max_decays:
            break
        # the standard error falls as 1/sqrt(n): aim just past the target
        need = int(min(max_decays - n, max(chunk, n * ((worst / tol) ** 2 * 1.05 - 1))))
        eng.run(PID_A, need, seed)
        n += need
    eng.sync()
    return org, sig, n, time.perf_counter() - t0, worst <= tol


def organ_dose_with_fallback(eng, net, prob, n_lo, seed, bias, tol=0.01, max_decays=10 ** 10,
                             ws=None):
    """Denoised organ doses with the Monte Carlo judge and fallback described
    in the module docstring.  Returns a dict with the organ values, the source
    of each ('denoiser' or 'mc'), decays and seconds."""
    eng.set_problem(PID_A, prob)
    eng.set_problem(PID_B, prob)
    if ws is None:
        ws = DN.Workspace(eng, prob.shape, train=False)
    eng.sync()
    t0 = time.perf_counter()
    half = n_lo // 2
    map_a = _run_map(eng, PID_A, half, seed)
    map_b = _run_map(eng, PID_B, half, seed)
    x_a = B.nmd_organ_mean_map(eng.ctx, PID_A, denoise_map(eng, net, PID_A, prob, map_a, ws),
                               prob.n_organs)
    x_b = B.nmd_organ_mean_map(eng.ctx, PID_B, denoise_map(eng, net, PID_B, prob, map_b, ws),
                               prob.n_organs)
    m_a, _, s_a = eng.organs(PID_A)
    m_b, _, s_b = eng.organs(PID_B)
    t_dn = time.perf_counter() - t0
    x = 0.5 * (x_a + x_b)
    mc = 0.5 * (m_a + m_b)
    sigma = _organ_sigma(s_a, s_b, m_a, m_b)
    delta = np.abs(x_a - x_b) / np.maximum(2 * x, 1e-300)
    est = np.sqrt(delta ** 2 + np.asarray(bias) ** 2)
    judged = np.abs(x - mc) <= 3 * sigma
    accept = (est <= tol) & judged
    n = 2 * half
    out = x.copy()
    src = np.where(accept, "denoiser", "mc")
    reached = True
    if not accept.all():
        while True:
            m_a, _, s_a = eng.organs(PID_A)
            m_b, _, s_b = eng.organs(PID_B)
            mc = 0.5 * (m_a + m_b)
            rel = 2 * _organ_sigma(s_a, s_b, m_a, m_b) / np.maximum(mc, 1e-300)
            worst = float(np.max(rel[~accept]))
            if worst <= tol or n >= max_decays:
                reached = worst <= tol
                break
            need = int(min(max_decays - n, max(2 * 10 ** 7, n * ((worst / tol) ** 2 * 1.05 - 1))))
            eng.run(PID_A, need // 2, seed)
            eng.run(PID_B, need // 2, seed)
            n += 2 * (need // 2)
        out[~accept] = mc[~accept]
    eng.sync()
    return {"organ": out, "source": src.tolist(), "estimated_error": est.tolist(),
            "judged": judged.tolist(), "mc_sigma": sigma.tolist(), "decays": int(n),
            "seconds": time.perf_counter() - t0, "seconds_denoiser_stage": t_dn,
            "reached": bool(reached)}


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="Train the dose denoiser on engine-generated data")
    ap.add_argument("--train-seeds", type=int, nargs=2, default=(10000, 10064))
    ap.add_argument("--eval-seeds", type=int, nargs=2, default=(20000, 20008))
    ap.add_argument("--n-lo", type=float, default=1e7)
    ap.add_argument("--n-hi", type=float, default=1e9)
    ap.add_argument("--boxes", type=int, default=4)
    ap.add_argument("--box", type=int, nargs=3, default=(160, 128, 128))
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight-floor", type=float, default=0.0,
                    help="loss weight 1/max(target, floor); 0 = plain MSE")
    ap.add_argument("--organ-boxes", type=float, default=0.0,
                    help="fraction of boxes centred on an organ voxel")
    ap.add_argument("--out", default="denoiser_weights.npz")
    ap.add_argument("--report", default="denoiser_report.json")
    a = ap.parse_args(argv)
    eng = B.Engine(0)
    net = DN.UNet(eng, seed=1)
    rng = np.random.default_rng(a.train_seeds[0])
    log = lambda m: print(m, flush=True)  # noqa: E731
    samples = make_samples(eng, range(*a.train_seeds), int(a.n_lo), int(a.n_hi), tuple(a.box),
                           a.boxes, rng, log=log, organ_fraction=a.organ_boxes)
    hist = train(eng, net, samples, a.steps, a.lr, log=log, weight_floor=a.weight_floor)
    del samples
    rows = evaluate(eng, net, range(*a.eval_seeds), int(a.n_lo), int(a.n_hi), log=log)
    bias = bias_table(rows)
    net.save(a.out, bias=bias)
    with open(a.report, "w") as f:
        json.dump({"history": hist, "eval": rows, "bias": bias.tolist(), "args": vars(a)}, f)
    log("saved %s and %s" % (a.out, a.report))


if __name__ == "__main__":
    main()
