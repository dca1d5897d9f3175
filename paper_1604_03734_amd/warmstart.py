"""Learned warm start of the primal-dual solver.

A small 3-D convolutional network (three 3x3x3 layers, 2 -> 16 -> 16 -> 1,
ReLU; BF16 MFMA kernels with FP32 accumulation in libdenser) maps the fused
TSDF of a block and its one-voxel halo, with the fusion weight as a second
channel, to one output field.  The primal-dual gap is governed by the dual
variable: starting from the exact minimiser u* with p = 0 takes as many
iterations as starting from zero, while starting from the exact dual p*
converges in a few tens.  So the network's output is used as a dual
component: it runs once per axis a on tiles whose x axis is the volume's
axis a (the energy is unchanged by exchanging axes, so one network serves
all three), its centre output is p_a, p0 is projected onto the unit ball and
u0 = f (DN_WARM_DUAL).  The primal use (u0 = clamp(f + r, -1, 1),
p0 = P(grad u0 / delta), DN_WARM_PRIMAL) is kept for comparison.

It is trained on the GPU by the library's own forward/backward kernels on
(fused block, regularised block) pairs that the method itself produces:
seeded synthetic streets are fused and regularised for 1000 iterations, and
blocks with enough observed voxels are sampled.

The plain solver stays in charge: after K warm-started iterations the
relative gap is compared with the plain solver's after K iterations from
zero with the same steps; if it is more than twice that, the warm start is
discarded and the solve restarts from zero.  Either way the solve runs until
the requested gap.  The plain solver's gap after K comes from a stored
calibration (measured on the training streets for a table of step sizes and
written beside the weights), or, for steps the table does not hold, from a
plain run of K iterations on the volume itself.

This module only sequences calls into the library (and uses torch for
device buffers); every computation runs in the HIP kernels.
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import denser as D

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart.npy")
CALIBRATION = os.path.join(HERE, "weights", "warmstart_calibration.json")
LAM = 0.5
# step sizes (tau, gamma) whose plain gap after K iterations is calibrated;
# sigma = 1 / (12 tau) for the fixed schedule
SCHEDULES = ((1.0 / np.sqrt(12.0), 0.0), (1.0 / np.sqrt(12.0), LAM), (0.02, 0.0), (0.03, 0.0), (0.05, 0.0),
             (0.1, 0.0))


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, a small last layer (r ~ 0 at start)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(D.NET_PARAMS, np.float32)
    p[0:864] = rng.normal(0, np.sqrt(2.0 / 54), 864)
    p[880:7792] = rng.normal(0, np.sqrt(2.0 / 432), 6912)
    p[7808:8240] = rng.normal(0, 0.1 * np.sqrt(1.0 / 432), 432)
    return p


def load_default_weights():
    if not os.path.exists(DEFAULT_WEIGHTS):
        return None
    w = np.load(DEFAULT_WEIGHTS, allow_pickle=False).astype(np.float32)
    if w.shape != (D.NET_PARAMS,):
        return None
    return w


def load_calibration(path=CALIBRATION):
    if not os.path.exists(path):
        return None
    import json
    with open(path) as f:
        return json.load(f)


def calibrated_gap(tau, gamma, k, cal=None):
    """The stored plain relative gap after k iterations at (tau, gamma), or
    None if the calibration does not hold these steps."""
    cal = load_calibration() if cal is None else cal
    if not cal or cal.get("k") != k:
        return None
    for e in cal["entries"]:
        if abs(e["tau"] - tau) <= 1e-9 * tau and abs(e["gamma"] - gamma) <= 1e-12:
            return e["plain_rel_gap"]
    return None


def calibrate(seeds=tuple(range(1001, 1007)), k=100, schedules=SCHEDULES, length=100.0, n_frames=100):
    """Relative gap of the plain solver (from zero) after k iterations on
    each seeded street, for each schedule; the largest over the streets is
    the one the fallback compares with."""
    import scenes
    out = {"k": k, "lambda": LAM, "streets": list(seeds), "entries": []}
    gaps = {sch: [] for sch in schedules}
    for s in seeds:
        vol = fuse_frames(scenes.frames_street(length, n_frames, seed=s, config_id=5))
        for tau, gamma in schedules:
            st = vol.regularize(D.reg_params(LAM, tau, 1.0 / (12.0 * tau), iters=k, gamma=gamma))
            gaps[(tau, gamma)].append(float(st.rel_gap))
        vol.close()
    for (tau, gamma), g in gaps.items():
        out["entries"].append({"tau": tau, "gamma": gamma, "plain_rel_gap": max(g), "per_street": g})
    return out


def fuse_frames(frames, max_blocks=16384):
    import torch
    cam = frames.camera
    K = D.intrinsics(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height)
    vol = D.Volume(frames.voxel_size, frames.mu, frames.max_depth, max_blocks, 16, 1024,
                   max_points=cam.width * cam.height)
    for d, T in zip(frames.depths, frames.poses):
        vol.integrate(torch.from_numpy(d).cuda(), K, T)
    return vol


def _to_tile_order(a, perm):
    """Block fields [n][512] (x fastest) in the centre order of a tile whose
    x axis is the volume's axis `perm` (the order dn_net_gather uses)."""
    b = a.reshape(-1, 8, 8, 8)             # [n][z][y][x]
    if perm == 1:
        b = b.permute(0, 1, 3, 2)
    elif perm == 2:
        b = b.permute(0, 3, 2, 1)
    return b.reshape(-1, 512).contiguous()


def make_pairs(seeds=(1001, 1002), n_pairs=5000, iters=1000, min_omega=64, length=100.0,
               n_frames=100, sample_seed=0, kind=1):
    """Training pairs on the device from seeded streets, fused and then
    regularised for `iters` iterations.
    kind 1 (dual): for every sampled block and axis a, the tile whose x axis
    is a and the dual component p_a of the regularised block (mask m_a).
    kind 0 (primal): the tile and the regularised u (mask Omega)."""
    import torch
    import scenes
    tiles_l, tgt_l, msk_l = [], [], []
    per = int(np.ceil(n_pairs / len(seeds)))
    rng = np.random.default_rng(sample_seed)
    for s in seeds:
        fr = scenes.frames_street(length, n_frames, seed=s, config_id=5)
        vol = fuse_frames(fr)
        vol.regularize(D.reg_params(LAM, iters=iters, kernel=D.DN_K_FUSED, gamma=LAM if kind == 1 else 0.0))
        w = vol.extract(D.DN_X_W)
        u = vol.extract(D.DN_X_U)
        p = vol.extract(D.DN_X_P)
        em = vol.extract(D.DN_X_EMASK)
        cnt = (w > 0).sum(1)
        cand = torch.nonzero(cnt >= min_omega).flatten().cpu().numpy()
        pick = np.sort(rng.choice(cand, size=min(per, len(cand)), replace=False)).astype(np.int32)
        blocks = torch.from_numpy(pick).cuda()
        bl = blocks.long()
        for a in (range(3) if kind == 1 else range(1)):
            tiles = torch.empty((len(pick), 2, 10, 10, 10), device="cuda")
            vol.net_gather(blocks, tiles, perm=a)
            tiles_l.append(tiles)
            if kind == 1:
                tgt_l.append(_to_tile_order(p[a][bl], a))
                msk_l.append(_to_tile_order(((em[bl] >> (a + 1)) & 1).float(), a))
            else:
                tgt_l.append(u[bl].contiguous())
                msk_l.append((w[bl] > 0).float().contiguous())
        torch.cuda.synchronize()
        vol.close()
    return torch.cat(tiles_l).contiguous(), torch.cat(tgt_l).contiguous(), torch.cat(msk_l).contiguous()


def train(tiles, targets, masks, epochs=60, batch=1024, lr=4e-3, seed=0, params=None, log=None, kind=1,
          lr_final=None):
    """Adam on the masked squared error (of r for kind 1, of f + r for
    kind 0), all on the GPU with the library's kernels.  With lr_final the
    step size follows a cosine from lr down to lr_final over the run."""
    import torch
    n = tiles.shape[0]
    p = torch.from_numpy(init_params(seed) if params is None else params).cuda().contiguous()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.empty_like(p)
    rng = np.random.default_rng(seed)
    step = 0
    hist = []
    total = epochs * max(1, (n - batch) // batch + 1)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        tot, nb = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            loss = D.net_loss_grad(tiles[idx].contiguous(), p, targets[idx].contiguous(),
                                   masks[idx].contiguous(), g, kind=kind)
            a = lr if lr_final is None else lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * step / total))
            step += 1
            D.net_adam(p, g, m, v, a, step)
            tot += loss
            nb += 1
        hist.append(tot / max(1, nb))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    torch.cuda.synchronize()
    return p, hist


def warm_state(vol, params, mode=D.DN_WARM_DUAL, delta=0.1):
    import torch
    nb = vol.num_blocks
    u0 = torch.empty((nb, 512), device="cuda")
    p0 = torch.empty((3, nb, 512), device="cuda")
    vol.net_warm_start(params, u0, p0, mode=mode, delta=delta)
    return u0, p0


def solve_plain(vol, tol=1e-3, max_iters=20000, gap_every=10, gamma=0.0, kernel=D.DN_K_AUTO):
    return vol.regularize(D.reg_params(LAM, iters=max_iters, gap_every=gap_every, gap_tol=tol,
                                       kernel=kernel, gamma=gamma))


def solve_warm(vol, params, tol=1e-3, k=100, plain_rel_gap_at_k=None, delta=0.1, max_iters=20000,
               gap_every=10, gamma=0.0, kernel=D.DN_K_AUTO, tau0=None, mode=D.DN_WARM_DUAL, calibration=None):
    """Warm start, K iterations, the fallback test, then iterate to `tol`.
    plain_rel_gap_at_k: the plain solver's relative gap after K iterations
    at the same steps; None: the stored calibration's, else a plain run of
    K iterations on `vol` (counted in the time).  Returns a dict with
    iterations, timings, whether it fell back and where the reference came
    from."""
    import torch
    if not isinstance(params, torch.Tensor):
        params = torch.from_numpy(np.asarray(params, np.float32)).cuda()
    # a warm start needs smaller primal and larger dual steps (tau sigma = 1/12)
    tau = 1.0 / np.sqrt(12.0) if tau0 is None else tau0
    sigma = 1.0 / (12.0 * tau)
    t0 = time.time()
    source = "given"
    if plain_rel_gap_at_k is None:
        plain_rel_gap_at_k = calibrated_gap(tau, gamma, k, calibration)
        source = "calibration"
        if plain_rel_gap_at_k is None:
            ref = vol.regularize(D.reg_params(LAM, tau, sigma, iters=k, kernel=kernel, gamma=gamma))
            plain_rel_gap_at_k = ref.rel_gap
            source = "plain run"
    u0, p0 = warm_state(vol, params, mode, delta)
    st = vol.regularize(D.reg_params(LAM, tau, sigma, iters=k, gap_every=gap_every, gap_tol=tol,
                                     init=D.DN_INIT_GIVEN, kernel=kernel, gamma=gamma), u0, p0)
    out = {"k": k, "iters_warm": st.iters_run, "rel_gap_at_k": st.rel_gap, "fallback": False,
           "reference": source, "plain_rel_gap_at_k": plain_rel_gap_at_k}
    if st.converged:
        out.update(iters=st.iters_run, converged=True, rel_gap=st.rel_gap, seconds=time.time() - t0)
        return out
    if not (st.rel_gap <= 2.0 * plain_rel_gap_at_k):
        out["fallback"] = True
        st2 = solve_plain(vol, tol, max_iters, gap_every, gamma, kernel)
        out.update(iters=st.iters_run + st2.iters_run, converged=bool(st2.converged), rel_gap=st2.rel_gap,
                   seconds=time.time() - t0)
        return out
    st2 = vol.regularize(D.reg_params(LAM, tau, sigma, iters=max_iters - k, gap_every=gap_every, gap_tol=tol,
                                      init=D.DN_INIT_KEEP, kernel=kernel, gamma=gamma))
    out.update(iters=st.iters_run + st2.iters_run, converged=bool(st2.converged), rel_gap=st2.rel_gap,
               seconds=time.time() - t0)
    return out


def main():
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="train the warm-start network on the GPU")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--streets", type=int, default=6, help="training streets (seeds 1001, 1002, ...)")
    ap.add_argument("--pairs", type=int, default=48000, help="sampled blocks over all streets (x3 axes)")
    ap.add_argument("--epochs", type=int, default=800)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=5e-5)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--calibration-out", default=CALIBRATION)
    ap.add_argument("--calibrate-only", action="store_true",
                    help="only measure the plain solver's gap after K on the training streets")
    args = ap.parse_args()
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    seeds = tuple(1001 + i for i in range(args.streets))

    def write_calibration():
        import json
        t = time.time()
        cal = calibrate(seeds)
        with open(args.calibration_out, "w") as f:
            json.dump(cal, f, indent=1)
        log(f"calibration of the fallback in {time.time() - t:.1f}s: " +
            ", ".join(f"tau {e['tau']:.3f} gamma {e['gamma']}: {e['plain_rel_gap']:.3e}" for e in cal["entries"]))

    if args.calibrate_only:
        write_calibration()
        return
    t0 = time.time()
    tiles, tgt, msk = make_pairs(seeds=seeds, n_pairs=args.pairs)
    log(f"{tiles.shape[0]} pairs in {time.time() - t0:.1f}s")
    t1 = time.time()
    p, hist = train(tiles, tgt, msk, epochs=args.epochs, lr=args.lr, batch=args.batch, log=log,
                    lr_final=args.lr_final)
    log(f"trained in {time.time() - t1:.1f}s")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, p.cpu().numpy().astype(np.float32), allow_pickle=False)
    write_calibration()
    print(args.out)


if __name__ == "__main__":
    main()
