#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X: street-scale fusion into hashed
8^3 blocks followed by Omega-masked TV primal-dual regularisation.

One step (timed, inputs already resident in HBM):
  1. allocate + fuse 100 synthetic 1242x375 depth maps of a 100 m street
     (0.2 m voxels, mu = 0.6 m) into a block-hashed volume;
  2. lay out the fused street `--copies` times side by side (translated
     along x, no shared faces) in one volume, to reach the ~2e5-block map of
     the street-scale workload (the 100 m street alone holds ~5.8e3
     blocks), through the library's own block insertion;
  3. 500 Chambolle-Pock iterations (lambda 0.5, tau = sigma = 1/sqrt(12))
     with the final primal-dual gap in float64;
  4. extraction of the zero-crossing surface.
value = allocated voxels x iterations / step time (voxel-iterations/s).

The JSON line also carries the roofline of the dominant kernel (the fused
iteration kernel, 48 algorithmic bytes per voxel-iteration, timed with HIP
events on the volume's stream), the FP64 CPU oracle timed on one street as
the CPU baseline, and the time to a relative gap of 1e-3 of the plain and
the warm-started solver.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

ALG_BYTES_PER_VOXEL_ITER = 48  # u, ubar, p(3), f, w read; p(3), u, ubar written (FP32)
ALG_BYTES_PER_VOXEL_ITER_16 = 28  # the same with u, ubar, p stored in 16 bits (f, w FP32)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--copies", type=int, default=35)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "fused256", "twopass"],
                    help="iteration kernel; with --workload batched: fused = the persistent kernel, "
                         "fused256 = one launch per iteration")
    ap.add_argument("--data-term", default="l2", choices=["l2", "l1"],
                    help="quadratic data term (the paper's) or the TV-L1 variant")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"],
                    help="storage of u, ubar, p (arithmetic is FP32 in every case)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-gap", action="store_true", help="skip the time-to-gap comparison")
    ap.add_argument("--workload", default="street", choices=["street", "batched"],
                    help="street: the street-scale map (default); batched: 64 uneven sub-maps "
                         "in one HIP graph")
    ap.add_argument("--submaps", type=int, default=64)
    ap.add_argument("--calib-copy", action="store_true",
                    help="only copy 1 GiB device to device (HBM counter calibration) and exit")
    ap.add_argument("--profile", action="store_true",
                    help="short run for profilers: no CPU baseline, no time-to-gap")
    ap.add_argument("--net-only", action="store_true",
                    help="only the network section (warm-start inference on the street map and "
                         "training steps), one JSON line, for profilers")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_digest(names=("cp_kernel.h", "regularize.hip")):
    """Digest of the sources of the iteration kernels."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1604_03734_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


TRAFFIC_FILES = {
    ("street", "f32"): ("cp_fused_street35_traffic.json", ("cp_kernel.h", "regularize.hip")),
    ("street", "f16"): ("cp_fused_street35_f16_traffic.json", ("cp_kernel.h", "regularize.hip")),
    ("street", "bf16"): ("cp_fused_street35_bf16_traffic.json", ("cp_kernel.h", "regularize.hip")),
    # by the variant that ran: the persistent kernel, one launch per iteration
    ("batched", "f32"): ({257: "cp_persistent_batched64_traffic.json", 1: "cp_batch_step_batched64_traffic.json"},
                         ("cp_kernel.h", "batch.hip")),
}


def load_traffic(nvox, workload, storage, kernel_id, layout=None):
    """Bytes leaving L2 per launch of the iteration kernel, from the
    committed counter summary, if it was taken on the current kernel source
    and on the kernel variant (and, where the summary records it, the block
    order) that ran (else None)."""
    entry = TRAFFIC_FILES.get((workload, storage))
    if entry is None:
        return None
    name, srcs = entry
    if isinstance(name, dict):
        name = name.get(kernel_id)
        if name is None:
            return None
    p = os.path.join(ROOT, "profiles", name)
    try:
        with open(p) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("source_digest") != src_digest(srcs) or t.get("kernel_id") != kernel_id:
        return None
    if "layout_used" in t and layout is not None and t["layout_used"] != layout:
        return None
    return t["bytes_per_voxel_iter"] * nvox


class Workload:
    def __init__(self, args):
        import torch
        import scenes
        from paper_1604_03734_amd import denser as D
        self.D, self.torch, self.args = D, torch, args
        t0 = time.time()
        self.fr = scenes.frames_c2(0, n_frames=args.frames)
        log(f"generated {len(self.fr.depths)} depth maps in {time.time() - t0:.1f}s")
        cam = self.fr.camera
        self.K = D.intrinsics(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height)
        self.depths = [torch.from_numpy(d).cuda() for d in self.fr.depths]
        self.street = D.Volume(self.fr.voxel_size, self.fr.mu, self.fr.max_depth, 16384, 16, 1024,
                               max_points=cam.width * cam.height)
        # the map is built from keys (no sensor input)
        self.big = D.Volume(self.fr.voxel_size, self.fr.mu, self.fr.max_depth, 1 << 18, 19, 8192,
                            max_points=0, max_candidates=1 << 18)
        self.kernel = {"auto": D.DN_K_AUTO, "fused": D.DN_K_FUSED, "fused256": D.DN_K_FUSED256,
                       "twopass": D.DN_K_TWOPASS}[args.kernel]
        # The HIP runtime takes a one-time stall of 30-70 ms once a process
        # has launched a few thousand kernels (measured: one slow batch of
        # launches, then none); fusing the street a few times here, before
        # anything is timed, keeps it out of the steady-state steps.
        for _ in range(4):
            self.fuse_street()
        torch.cuda.synchronize()

    def fuse_street(self):
        self.street.clear()
        for d, T in zip(self.depths, self.fr.poses):
            self.street.alloc_blocks(d, self.K, T)
            self.street.fuse_depth(d, self.K, T)

    def build_map(self):
        """Translated copies of the fused street in one volume, each copy's
        blocks allocated in the order fusion allocated the street's (one
        order-keeping insertion), copy after copy."""
        D, torch = self.D, self.torch
        c = self.street.extract(D.DN_X_COORDS).long()      # the street's allocation order
        f = self.street.extract(D.DN_X_F)
        w = self.street.extract(D.DN_X_W)
        width = int((c[:, 0].max() - c[:, 0].min()).item()) + 3
        k = self.args.copies
        shift = torch.zeros((k, 1, 3), dtype=torch.long, device=c.device)
        shift[:, 0, 0] = torch.arange(k, device=c.device) * width
        coords = (c[None] + shift).reshape(-1, 3).to(torch.int32).contiguous()
        self.big.clear()
        self.big.insert_blocks(coords, keep_order=True)
        self.big.load_fused(f.repeat(k, 1).contiguous(), w.repeat(k, 1).contiguous())

    def step(self):
        D = self.D
        self.fuse_street()
        self.build_map()
        storage = {"f32": D.DN_F32, "f16": D.DN_F16, "bf16": D.DN_BF16}[self.args.storage]
        st = self.big.regularize(D.reg_params(0.5, iters=self.args.iters, gap_every=0, kernel=self.kernel,
                                              storage=storage, refine_every=50,
                                              data_term=D.DN_DATA_L1 if getattr(self.args, "data_term", "l2") == "l1" else 0))
        pts = self.big.extract(D.DN_X_SURFACE)
        return st, pts.shape[0]


class BatchedWorkload(Workload):
    """64 sub-maps with block counts drawn log-uniform in [1e3, 5e4]; each is
    a street segment: the n_i blocks nearest the start of a row of
    translated copies of the fused street.  A segment's blocks are
    allocated in the order the fused street allocated them (copy after
    copy; one order-keeping insertion), so its block pool holds them in
    allocation order, as a map built by fusion does.  All regularised
    together for 300 iterations in one HIP graph (the persistent kernel or
    one launch per iteration, autotuned)."""

    def __init__(self, args, base=None):
        if base is None:
            super().__init__(args)
        else:
            # share the generated frames and the fused street of a street workload
            self.D, self.torch, self.args = base.D, base.torch, args
            self.fr, self.K, self.depths, self.street = base.fr, base.K, base.depths, base.street
            self.big, self.kernel = base.big, base.kernel
        import scenes
        self.counts = scenes.c4_block_counts(args.submaps, seed=0)
        # the tuner's choice, or the persistent kernel / one launch per iteration
        self.batch_kernel = {"auto": self.D.DN_K_AUTO, "fused": self.D.DN_K_FUSED,
                             "fused256": self.D.DN_K_FUSED256}.get(getattr(args, "kernel", "auto"), self.D.DN_K_AUTO)
        self.subs = []
        for n in self.counts:
            self.subs.append(self.D.Volume(self.fr.voxel_size, self.fr.mu, self.fr.max_depth, int(n),
                                           max(10, int(np.ceil(np.log2(n))) + 1), 4096, max_points=0,
                                           state16=False))
        if base is None:
            self.fuse_street()
        self._layout()

    def _layout(self):
        D, torch = self.D, self.torch
        c = self.street.extract(D.DN_X_COORDS).long()      # in the street's allocation order
        f = self.street.extract(D.DN_X_F)
        w = self.street.extract(D.DN_X_W)
        zlen = int((c[:, 2].max() - c[:, 2].min()).item()) + 3
        off = 1 << 20
        self.parts = []
        for vol, n in zip(self.subs, self.counts):
            reps = int(np.ceil(n / c.shape[0]))
            shift = torch.zeros((reps, 1, 3), dtype=torch.long, device=c.device)
            shift[:, 0, 2] = torch.arange(reps, device=c.device) * zlen
            cc = (c[None] + shift).reshape(-1, 3)
            # the segment: the n blocks with the smallest z (ties by x, y),
            # taken in allocation order (copy, then the street's pool order)
            key = ((cc[:, 2] + off) << 42) | ((cc[:, 0] + off) << 21) | (cc[:, 1] + off)
            sel = torch.sort(torch.argsort(key)[: int(n)]).values
            vol.clear()
            vol.insert_blocks(cc[sel].to(torch.int32).contiguous(), keep_order=True)
            src = sel % c.shape[0]
            self.parts.append((f[src].contiguous(), w[src].contiguous()))

    def step(self):
        D = self.D
        for vol, (f, w) in zip(self.subs, self.parts):
            vol.load_fused(f, w)
        stats = D.regularize_batch(self.subs, D.reg_params(0.5, iters=self.args.iters, kernel=self.batch_kernel))
        return stats[0], 0

    def voxels(self):
        return int(sum(v.num_blocks for v in self.subs)) * 512


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, cp_iters=20):
    """The FP64 oracle on the host's cores on a bounded sample of the same
    step: allocation + fusion of the 100 depth maps of the street, then
    cp_iters iterations over the whole map of translated copies (the same
    blocks the GPU regularises); the step rate is extrapolated to the
    step's 500 iterations."""
    import oracle
    D = wl.D
    fr = wl.fr
    cam = fr.camera
    K4 = [cam.fx, cam.fy, cam.cx, cam.cy]
    nt = oracle.nthreads_default()
    t0 = time.time()
    ov = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 16384, 16, 1024)
    for d, T in zip(fr.depths, fr.poses):
        ov.alloc(d, K4, T)
        ov.fuse(d, K4, T, nthreads=nt)
    t_fuse = time.time() - t0
    # the map: the GPU map's keys (the same translated copies), f and w
    coords = wl.big.extract(D.DN_X_COORDS).cpu().numpy()
    f = wl.big.extract(D.DN_X_F).cpu().numpy().astype(np.float64)
    w = wl.big.extract(D.DN_X_W).cpu().numpy().astype(np.float64)
    big = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, len(coords), 19, 8192)
    big.insert(coords)
    u = np.zeros_like(f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
    t1 = time.time()
    oracle.cp(big.nbr, f, w, u, ub, p, cp_iters, 0.5, 12 ** -0.5, 12 ** -0.5, 1.0, nthreads=nt)
    t_cp = time.time() - t1
    vox = len(coords) * 512
    iters = wl.args.iters
    t_step = t_fuse + t_cp * iters / cp_iters
    return {
        "value": vox * iters / t_step, "unit": "voxel-iterations/s", "cores": nt,
        "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
        "sample": f"alloc+fuse of the {len(fr.depths)} street frames ({t_fuse:.1f}s) + {cp_iters} iterations "
                  f"over the whole {len(coords)}-block map ({t_cp:.1f}s), extrapolated to {iters} iterations",
        "cp_only_voxel_iters_per_s": vox * cp_iters / t_cp,
    }


def accuracy(wl, iters=500):
    """Synthetic analogue of the paper's error statistics (Section V,
    Tables III and IV): distance of the zero-crossing surface of the street
    to the analytic scene and area of its mesh, before (u = f) and after
    regularisation.  Points inside a solid box are counted apart (their
    distance to the nearest face is capped by the box's half thickness), and
    the median / 75th percentile are also given over the points outside."""
    import scenes
    D, torch = wl.D, wl.torch
    vol = wl.street
    boxes = scenes.scene_street(100.0, 0, 2)
    f = vol.extract(D.DN_X_F)
    out = {}
    for name, prm, u0 in (("raw", D.reg_params(0.5, iters=0, init=D.DN_INIT_GIVEN), f),
                          ("regularised", D.reg_params(0.5, iters=iters, kernel=D.DN_K_AUTO), None)):
        vol.regularize(prm, u0=u0)
        pts = vol.extract(D.DN_X_SURFACE).cpu().numpy()
        d = scenes.distance_to_scene(pts, boxes) * 100.0
        ins = scenes.inside_scene(pts, boxes)
        do = d[~ins]
        area, ntri = vol.mesh_area()
        out[name] = {"points": int(len(pts)), "inside_share": float(ins.mean()),
                     "median_cm": float(np.median(d)), "p75_cm": float(np.percentile(d, 75)),
                     "mean_cm": float(d.mean()),
                     "outside_points": int(len(do)), "outside_median_cm": float(np.median(do)),
                     "outside_p75_cm": float(np.percentile(do, 75)),
                     "mesh_area_m2": area, "mesh_triangles": ntri}
    r, g = out["raw"], out["regularised"]
    out["median_change"] = g["median_cm"] / r["median_cm"] - 1.0
    out["p75_change"] = g["p75_cm"] / r["p75_cm"] - 1.0
    out["outside_median_change"] = g["outside_median_cm"] / r["outside_median_cm"] - 1.0
    out["outside_p75_change"] = g["outside_p75_cm"] / r["outside_p75_cm"] - 1.0
    out["points_change"] = g["points"] / r["points"] - 1.0
    out["area_change"] = g["mesh_area_m2"] / r["mesh_area_m2"] - 1.0
    return out


def time_to_gap(wl, tol=1e-3, k=100):
    """Wall time to relative gap <= tol on the street map, from zero (plain)
    and from the learned warm start (network inference + iterations, with
    the fallback to a cold start), both with their gap checks (every 10
    iterations).  For the configured fixed steps (tau = sigma = 1/sqrt(12)),
    for the accelerated variant (gamma = lambda), and with each solver at its
    fastest step ratio among the same candidates.  The fallback compares the
    warm gap after k iterations with the plain solver's after k iterations
    at the same steps, taken from the calibration stored with the weights
    (measured on the training streets); for the first two schedules the
    solve is also timed with that reference measured by a plain run of k
    iterations on the map itself, counted in the warm time."""
    D = wl.D
    torch = wl.torch
    from paper_1604_03734_amd import warmstart
    w = warmstart.load_default_weights()
    wt = torch.from_numpy(w).cuda() if w is not None else None
    out = {"tol": tol, "k": k, "weights": "paper_1604_03734_amd/weights/warmstart.npy" if w is not None else None,
           "calibration": "paper_1604_03734_amd/weights/warmstart_calibration.json"
           if warmstart.load_calibration() is not None else None}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.time()
        r = fn()
        torch.cuda.synchronize()
        return r, time.time() - t0

    def warm(tau, gam, reference=None):
        return timed(lambda: warmstart.solve_warm(wl.big, wt, tol=tol, k=k, gamma=gam, tau0=tau,
                                                  plain_rel_gap_at_k=reference))

    t0 = 1.0 / np.sqrt(12.0)
    for name, gam in (("fixed_steps", 0.0), ("accelerated", 0.5)):
        r = {}
        st, r["plain_s"] = timed(lambda: warmstart.solve_plain(wl.big, tol, gamma=gam))
        r["plain_iters"] = st.iters_run
        r["plain_converged"] = bool(st.converged)
        if wt is not None:
            res, warm_s = warm(t0, gam)
            r.update(warm_s=warm_s, warm_iters=res["iters"], warm_converged=res["converged"],
                     warm_fallback=res["fallback"], fallback_reference=res["reference"],
                     speedup=r["plain_s"] / warm_s)
            ref, ref_s = timed(lambda: wl.big.regularize(D.reg_params(0.5, t0, 1.0 / (12.0 * t0), iters=k,
                                                                      gamma=gam)))
            res2, warm2_s = warm(t0, gam, ref.rel_gap)
            r["with_reference_run"] = {"warm_s": warm2_s + ref_s, "reference_s": ref_s,
                                       "warm_iters": res2["iters"], "warm_fallback": res2["fallback"],
                                       "speedup": r["plain_s"] / (warm2_s + ref_s)}
        out[name] = r
    # each solver at its best step ratio: tau from the same candidates,
    # sigma = 1 / (12 tau), both with the fixed schedule
    if wt is not None:
        cand = (0.02, 0.03, 0.05, 0.1, t0)
        plain, warm_r = {}, {}
        for tau in cand:
            st, ps = timed(lambda: wl.big.regularize(D.reg_params(0.5, tau, 1.0 / (12.0 * tau), iters=20000,
                                                                  gap_every=10, gap_tol=tol)))
            plain[tau] = (ps, st.iters_run, bool(st.converged))
            res, ws = warm(tau, 0.0)
            warm_r[tau] = (ws, res["iters"], bool(res["converged"]), bool(res["fallback"]), res["reference"])
        bp = min((v[0], t) for t, v in plain.items() if v[2])[1]
        bw = min((v[0], t) for t, v in warm_r.items() if v[2])[1]
        out["best_steps"] = {"tau_candidates": list(cand),
                             "plain_tau": bp, "plain_s": plain[bp][0], "plain_iters": plain[bp][1],
                             "warm_tau": bw, "warm_s": warm_r[bw][0], "warm_iters": warm_r[bw][1],
                             "warm_fallback": warm_r[bw][3], "fallback_reference": warm_r[bw][4],
                             "speedup": plain[bp][0] / warm_r[bw][0]}
    return out


def fusion_scaling(wl):
    """Per-frame cost of depth fusion (Eq. 1) into the fused street and into
    the whole map (35 copies, the street is one of them): fusion culls the
    blocks out of view, so the map costs the street's visible blocks plus
    one cheap test per block.  Changes the f/w of both volumes (runs last)."""
    torch = wl.torch
    out = {}
    for name, vol in (("street", wl.street), ("map", wl.big)):
        vol.fuse_depth(wl.depths[0], wl.K, wl.fr.poses[0])
        torch.cuda.synchronize()
        t0 = time.time()
        for d, T in zip(wl.depths, wl.fr.poses):
            vol.fuse_depth(d, wl.K, T)
        torch.cuda.synchronize()
        out[name] = {"blocks": vol.num_blocks, "ms_per_frame": 1000.0 * (time.time() - t0) / len(wl.depths)}
    return out


def x1_mixed_precision(wl, fp32_ms, iters=100):
    """FP16 / BF16 storage of u, ubar, p (FP32 arithmetic, stochastic
    rounding, FP32 refinement sweep every 50 iterations): time per iteration
    on the street map with its roofline (28 algorithmic bytes per
    voxel-iteration; the loop average includes the sweeps), and the error
    against the FP64 oracle on the small scene after 200 iterations."""
    import oracle
    import scenes
    D = wl.D
    nvox = wl.big.num_blocks * 512
    out = {}
    for name, s in (("f16", D.DN_F16), ("bf16", D.DN_BF16)):
        prm = D.reg_params(0.5, iters=iters, storage=s, refine_every=50)
        wl.big.regularize(prm)                    # the tuner's first call
        st = wl.big.regularize(prm)
        ms = st.ms_loop / iters
        ach = ALG_BYTES_PER_VOXEL_ITER_16 * nvox / (ms / 1000.0) / 1e9
        out[name] = {"ms_per_iter": ms, "speedup_vs_f32": fp32_ms / ms,
                     "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": ach / HBM_PEAK_GBS,
                                  "traffic": load_traffic(nvox, "street", name, st.kernel_used),
                                  "alg_bytes_per_launch": ALG_BYTES_PER_VOXEL_ITER_16 * nvox}}
    fr = scenes.frames_c1(0)
    cam = fr.camera
    K4 = [cam.fx, cam.fy, cam.cx, cam.cy]
    ov = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 8192, 12, 256)
    gv = D.Volume(fr.voxel_size, fr.mu, fr.max_depth, 8192, 12, 256, max_points=cam.width * cam.height)
    for d, T in zip(fr.depths, fr.poses):
        ov.integrate(d, K4, T)
        gv.integrate(wl.torch.from_numpy(d).cuda(), D.intrinsics(*K4, cam.width, cam.height), T)
    u = np.zeros_like(ov.f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
    oracle.cp(ov.nbr, ov.f, ov.w, u, ub, p, 200, 0.5, 12 ** -0.5, 12 ** -0.5, 1.0)
    om = ov.w > 0
    band = om & (np.abs(u) < 1.0)          # the TSDF band, away from the truncation
    E, Dd = oracle.energy(ov.nbr, ov.f, ov.w, u, p, 0.5)
    for name, s in (("f32", D.DN_F32), ("f16", D.DN_F16), ("bf16", D.DN_BF16)):
        st = gv.regularize(D.reg_params(0.5, iters=200, storage=s, refine_every=50))
        err = np.abs(gv.extract(D.DN_X_U).cpu().numpy().astype(np.float64) - u)
        e, eb = err[om], err[band]
        out.setdefault(name, {})["error_vs_oracle"] = {
            "max": float(e.max()), "median": float(np.median(e)),
            "band_max": float(eb.max()), "band_median": float(np.median(eb)),
            "rel_gap": float(st.rel_gap), "oracle_rel_gap": float((E - Dd) / E),
            "scene": "small scene (4 maps 320x96), 200 iterations; band: voxels of Omega with |u| < 1"}
    gv.close()
    return out


# variant codes of the batched solver (kernel_used // 100)
BATCH_KERNELS = {257: "k_cp_persistent_lean", 256: "k_cp_persistent<256>", 512: "k_cp_persistent<512>",
                 1: "k_cp_batch_step (one launch per iteration)"}


def batched_run(wl, submaps=64, iters=300, steps=2):
    """Batched sub-maps in the default run: 64 street segments with block
    counts log-uniform in [1e3, 5e4], regularised for 300 iterations in one
    HIP graph (persistent kernel or one launch per iteration, autotuned)."""
    import types
    D = wl.D
    bw = BatchedWorkload(types.SimpleNamespace(submaps=submaps, iters=iters), base=wl)
    st, _ = bw.step()                                 # tuner + graph capture
    ms = []
    for _ in range(steps):
        st, _ = bw.step()
        ms.append(st.ms_loop / iters)
    nvox = bw.voxels()
    per = float(np.mean(ms))
    ach = ALG_BYTES_PER_VOXEL_ITER * nvox / (per / 1000.0) / 1e9
    kid = st.kernel_used // 100
    out = {"submaps": submaps, "blocks": nvox // 512, "voxels": nvox, "iters": iters,
           "ms_per_iter": per, "voxel_iters_per_s": nvox / (per / 1000.0),
           "kernel": BATCH_KERNELS.get(kid, "k_cp_persistent"),
           "wg_per_cu": st.kernel_used % 100,
           "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS,
                        "traffic": load_traffic(nvox, "batched", "f32", kid, st.layout_used),
                        "alg_bytes_per_launch": ALG_BYTES_PER_VOXEL_ITER * nvox}}
    for v in bw.subs:
        v.close()
    return out


def laser_throughput(wl, n_scans=10, rings=64, azimuth=1024):
    """Laser range fusion on the street (Section III-A's extension to laser
    sensors): synthetic 64 x 1024 scans every 10 m along the street, each
    allocated and fused into a fresh volume; returns per second of
    allocation + fusion (HIP events), inputs resident in HBM."""
    import scenes
    D, torch = wl.D, wl.torch
    boxes = scenes.scene_street(100.0, 0, 2)
    poses = [scenes.pose_translation(0.0, 0.0, 10.0 * k) for k in range(n_scans)]
    scans = [torch.from_numpy(scenes.laser_scan(boxes, T, k, n_rings=rings, n_azimuth=azimuth,
                                                 elev_deg=(-25.0, 3.0), max_range=50.0)).cuda()
             for k, T in enumerate(poses)]
    n_ret = rings * azimuth
    vol = D.Volume(wl.fr.voxel_size, wl.fr.mu, wl.fr.max_depth, 1 << 16, 18, 4096, max_points=n_ret,
                   max_observations=D.laser_observations_bound(n_ret, wl.fr.voxel_size, wl.fr.mu,
                                                              wl.fr.max_depth))
    for pts, T in zip(scans[:2], poses[:2]):
        vol.integrate_laser(pts, T)
    vol.clear()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for pts, T in zip(scans, poses):
        vol.integrate_laser(pts, T)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    n = sum(int(torch.isfinite(p[:, 0]).sum()) for p in scans)
    return {"scans": n_scans, "returns": n, "blocks": vol.num_blocks, "ms": ms,
            "returns_per_s": n / (ms / 1000.0)}


# dense matrix peak of the MI355X for bfloat16 operands (TFLOP/s)
MFMA_BF16_PEAK_TFLOPS = 2500.0
# useful multiply-adds x 2 of the network on one 10^3 tile: layers 1 and 2 on
# all 1000 voxels, layer 3 on the 512 centre voxels (inference) or on all
# 1000 (training forward)
NET_INFER_FLOP_PER_TILE = 2.0 * (1000 * 16 * 54 + 1000 * 16 * 432 + 512 * 432)
NET_FWD_FLOP_PER_TILE = 2.0 * (1000 * 16 * 54 + 1000 * 16 * 432 + 1000 * 432)
# training step: forward + weight gradients of 3 layers + input gradients of
# layers 3 and 2 (layer 1 needs none)
NET_TRAIN_FLOP_PER_TILE = 2 * NET_FWD_FLOP_PER_TILE + 2.0 * (1000 * 16 * 432 + 1000 * 432)


def net_rooflines(wl, reps=3, batch=1024, train_steps=20):
    """Matrix-core throughput of the network, timed with HIP events on the
    stream the library launches on: the dual warm start of the street map
    (gather pre-pass, one fused inference launch per axis, projection) and
    training steps (loss gradient + Adam) on batches of synthetic tiles."""
    D, torch = wl.D, wl.torch
    from paper_1604_03734_amd import warmstart
    w = warmstart.load_default_weights()
    prm = torch.from_numpy(w if w is not None else warmstart.init_params(0)).cuda()
    vol = wl.big
    nb = vol.num_blocks
    u0 = torch.empty((nb, 512), device="cuda")
    p0 = torch.empty((3, nb, 512), device="cuda")
    vol.net_warm_start(prm, u0, p0, mode=D.DN_WARM_DUAL)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        vol.net_warm_start(prm, u0, p0, mode=D.DN_WARM_DUAL)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tf = NET_INFER_FLOP_PER_TILE * nb * 3 / (ms / 1000.0) / 1e12
    out = {"inference": {"bound": "mfma", "what": f"dual warm start of the street map: {nb} tiles x 3 axes",
                         "ms": ms, "achieved": tf, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / MFMA_BF16_PEAK_TFLOPS, "flop_per_tile": NET_INFER_FLOP_PER_TILE}}
    del u0, p0
    g = torch.Generator(device="cpu").manual_seed(0)
    tiles = torch.randn((batch, 2, 10, 10, 10), generator=g).cuda()
    tgt = torch.randn((batch, 512), generator=g).cuda()
    msk = (torch.rand((batch, 512), generator=g) < 0.6).float().cuda()
    p = prm.clone()
    grad = torch.empty_like(p)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    D.net_loss_grad(tiles, p, tgt, msk, grad, kind=1)
    torch.cuda.synchronize()
    e0.record()
    for k in range(train_steps):
        D.net_loss_grad(tiles, p, tgt, msk, grad, kind=1, sync=False)
        D.net_adam(p, grad, m, v, 1e-4, k + 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / train_steps
    tf = NET_TRAIN_FLOP_PER_TILE * batch / (ms / 1000.0) / 1e12
    out["training"] = {"bound": "mfma", "what": f"loss gradient + Adam on {batch}-tile batches",
                       "ms_per_step": ms, "achieved": tf, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": tf / MFMA_BF16_PEAK_TFLOPS, "flop_per_tile": NET_TRAIN_FLOP_PER_TILE}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calib_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)  # one elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": x.numel() * 4}))
        return
    from paper_1604_03734_amd import denser as D
    D.lib()
    if args.profile:
        args.no_cpu = args.no_gap = True
    if args.workload == "batched":
        if "--iters" not in sys.argv:
            args.iters = 300
        args.no_gap = True
        wl = BatchedWorkload(args)
    else:
        wl = Workload(args)
    if args.net_only:
        wl.fuse_street()
        wl.build_map()
        print(json.dumps({"net_roofline": net_rooflines(wl)}), flush=True)
        return
    for i in range(args.warmup):
        st, npts = wl.step()
        torch.cuda.synchronize()
        log(f"warmup {i}: ms_loop {st.ms_loop:.1f}")
    torch.cuda.synchronize()
    times, loops = [], []
    t_all = time.time()
    for i in range(args.steps):
        t0 = time.time()
        st, npts = wl.step()
        torch.cuda.synchronize()
        times.append(time.time() - t0)
        loops.append(st.ms_loop / max(1, st.iters_run))
        log(f"step {i}: {times[-1]:.3f}s, loop {st.ms_loop:.1f} ms, rel_gap {st.rel_gap:.3e}, points {npts}")
    torch.cuda.synchronize()
    total = time.time() - t_all
    if args.workload == "batched":
        nvox = wl.voxels()
        nb = nvox // 512
    else:
        nb = wl.big.num_blocks
        nvox = nb * 512
    ms_step = 1000.0 * total / max(1, args.steps)
    value = nvox * args.iters / (ms_step / 1000.0)
    kern_ms = float(np.mean(loops))
    alg_bytes = ALG_BYTES_PER_VOXEL_ITER if args.storage == "f32" else ALG_BYTES_PER_VOXEL_ITER_16
    achieved = alg_bytes * nvox / (kern_ms / 1000.0) / 1e9
    kernel_id = st.kernel_used // 100 if args.workload == "batched" else st.kernel_used
    traffic = load_traffic(nvox, args.workload, args.storage, kernel_id,
                           st.layout_used if args.workload == "batched" else None)
    if args.workload == "batched":
        metric = f"voxel-iterations/s ({args.submaps} sub-maps, {args.iters} CP iterations, one HIP graph)"
        config = {"workload": f"batched sub-maps: {args.submaps} street segments with block counts "
                              "log-uniform in [1e3, 5e4] (0.2 m voxels), one HIP graph (persistent "
                              "kernel or one launch per iteration, autotuned)", "blocks": nb, "voxels": nvox,
                  "iters": args.iters, "lambda": 0.5}
        kname = BATCH_KERNELS.get(st.kernel_used // 100, "k_cp_persistent")
        kname += " (one CP iteration of every sub-map)"
    else:
        metric = f"voxel-iterations/s (fusion + {args.iters} CP iterations + gap + surface, street map)"
        config = {"workload": "street-scale plain method, FP32: 100 depth maps 1242x375 of a 100 m "
                              "synthetic street, 0.2 m voxels, mu 0.6 m, sigma 0.5 px, 5% invalid; "
                              f"map = {args.copies} translated copies of the fused street, blocks in its allocation order",
                  "blocks": nb, "voxels": nvox, "street_blocks": wl.street.num_blocks,
                  "iters": args.iters, "lambda": 0.5, "kernel": args.kernel, "storage": args.storage,
                  "data_term": args.data_term}
        kname = {1: "k_dual + k_primal", 2: "k_cp_fused", 3: "k_cp_fused256"}.get(st.kernel_used, "k_cp_fused")
        kname += " (one CP iteration)"
    line = {
        "metric": metric,
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "hbm", "kernel": kname,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes * nvox,
                     "avg_launch_ms": kern_ms},
        "cp_voxel_iters_per_s": nvox / (kern_ms / 1000.0),
    }
    if traffic is not None:
        # bytes leaving L2 per launch (rocprofv3 counters) over the live launch time
        line["roofline"]["traffic_gbs"] = traffic / (kern_ms / 1000.0) / 1e9
    if args.workload == "street":
        # the same rate per observed voxel (Omega: w > 0)
        n_omega = int((wl.big.extract(D.DN_X_W) > 0).sum().item())
        line["omega_voxels"] = n_omega
        line["cp_omega_voxel_iters_per_s"] = n_omega / (kern_ms / 1000.0)
    if args.workload == "batched":
        line["config"]["kernel_used"] = {"threads": 512 if st.kernel_used // 100 == 512 else 256,
                                         "lean": st.kernel_used // 100 == 257,
                                         "wg_per_cu": st.kernel_used % 100}
        line["config"]["layout_used"] = {"order": "pool" if st.layout_used & 1 else "morton",
                                         "xcd_chunks": not (st.layout_used & 2)}
    if args.workload == "street":
        names = {1: "twopass", 2: "fused512", 3: "fused256x2"}
        line["config"]["kernel_used"] = names.get(st.kernel_used, str(st.kernel_used))
        line["config"]["layout_used"] = {"order": "pool" if st.layout_used & 1 else "morton",
                                         "xcd_chunks": not (st.layout_used & 2)}
    if args.workload == "street":
        # the boundary takes device buffers; a caller with host depth maps
        # also pays their upload (pageable host memory here)
        torch.cuda.synchronize()
        t0 = time.time()
        up = [torch.from_numpy(d).cuda() for d in wl.fr.depths]
        torch.cuda.synchronize()
        h2d_ms = 1000.0 * (time.time() - t0)
        del up
        line["pcie_inclusive"] = {"h2d_ms_per_step": h2d_ms,
                                  "value": nvox * args.iters / ((ms_step + h2d_ms) / 1000.0)}
    if not args.no_cpu:
        log("timing the CPU oracle ...")
        line["cpu_baseline"] = cpu_baseline(wl)
    if args.workload == "street" and not args.profile:
        log("accuracy against the analytic scene ...")
        line["accuracy"] = accuracy(wl)
    if args.workload == "street" and not args.profile and args.storage == "f32":
        log("16-bit storage ...")
        line["x1"] = x1_mixed_precision(wl, kern_ms)
        log("batched sub-maps ...")
        line["batched"] = batched_run(wl)
    if args.workload == "street" and not args.profile:
        log("laser fusion ...")
        line["laser_fusion"] = laser_throughput(wl)
        log("network throughput ...")
        line["net_roofline"] = net_rooflines(wl)
    if not args.no_gap:
        log("time to gap ...")
        line["time_to_gap"] = time_to_gap(wl)
    if args.workload == "street" and not args.profile:
        log("fusion into the map ...")
        line["fusion_scaling"] = fusion_scaling(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
