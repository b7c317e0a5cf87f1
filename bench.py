"""Benchmark of libfock on one MI355X.

One step = one V_X application of one GPU's band-index share of a 512-Si-atom
cell (96^3 grid, L = 41.04 bohr, 1024 orbitals psi_j, 32 targets phi_k,
screened HSE kernel w = 0.106): 32768 pair Poisson solves, FP32 FFTs with FP64
accumulation over j.  Orbitals are synthetic (seeded random planewaves below
10 Ha, Loewdin-orthonormalised) and resident in HBM before timing starts.

Prints one JSON line: pairs/s, the roofline of the dominant kernel (timed with
HIP events on its own stream), the FP64 form on the same GPU and the FP64 CPU
oracle on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KSRC = ["paper_1905_01348_amd/csrc/vx.hip", "paper_1905_01348_amd/csrc/vx_passes.hpp",
        "paper_1905_01348_amd/csrc/fft.hpp"]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KSRC:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic HBM bytes per grid point per pair for each V_X kernel, storage
# of s bytes per complex value (8 for the FP32 path, 16 for FP64):
#   plane_fwd : read psi_j and phi_k, write the pair volume T   -> 3 s
#   pencil_z  : read and write T                                -> 2 s
#   plane_inv : read T and psi_j                                -> 2 s
#               + read and write the FP64 partial sum of phi_k once per
#                 batch of nj orbitals (16 B each way)          -> 32/nj
def algorithmic_bytes_per_pt(kernel, s, nj, multi_batch):
    if kernel == "vx_plane_fwd":
        return 3 * s
    if kernel == "vx_pencil_z":
        return 2 * s
    extra = (32.0 / nj) if multi_batch else (16.0 / nj)
    return 2 * s + extra


def cpu_baseline(psi_h, w, seconds):
    """The FP64 oracle as it stands, timed on a growing prefix of orbitals for target 0."""
    import numpy as np

    import oracle

    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    phi = psi_h[:1].astype(np.complex128)
    J, el = 4, 0.0
    while True:
        t0 = time.perf_counter()
        oracle.apply_vx(psi_h[:J], phi, w["n"], w["L"], "hse", 0.106, workers=cores)
        el = time.perf_counter() - t0
        if el >= seconds or J >= psi_h.shape[0]:
            break
        J = min(psi_h.shape[0], max(J * 2, int(J * seconds / max(el, 1e-3) * 1.05)))
    return {"value": J / el, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle.apply_vx on target phi_0 against psi_0..psi_{J - 1} "
                      f"({J} pairs of the same 96^3 workload, scipy.fft workers={cores}), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2", choices=["cfg1", "cfg2"])
    ap.add_argument("--prec", default="fp32acc64", choices=["fp32acc64", "fp32", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed FP64 steps for the comparison (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU oracle budget (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU ring pass is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1905_01348_amd import Context, fock

    w = synth.workload(args.workload)
    n, L, N, Nt = w["n"], w["L"], w["N"], w["n_targets"]
    nr = n ** 3
    log(f"[bench] generating {args.workload}: {N} orbitals on {n}^3 ...")
    t0 = time.time()
    in_dtype = np.complex128 if args.prec == "fp64" else np.complex64
    psi_h = synth.make_orbitals(w["seed"], n, L, N, dtype=in_dtype)
    log(f"[bench] generated in {time.time() - t0:.1f} s")
    dev = torch.device("cuda:0")
    P = torch.from_numpy(psi_h).to(dev)
    phi = P[:Nt]
    out = torch.empty((Nt, n, n, n), dtype=torch.complex128 if args.prec != "fp32" else torch.complex64, device=dev)
    ctx = Context(0)
    kw = dict(n=n, L=L, kernel="hse", omega=0.106, prec=args.prec, out=out)

    for i in range(args.warmup):
        ctx.apply_vx(P, phi, **kw)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    ctx.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.apply_vx(P, phi, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"[bench] {args.steps} steps in {el:.3f} s")
    pairs = N * Nt
    value = pairs * args.steps / el
    ms_per_step = 1e3 * el / args.steps

    # per-kernel durations over the timed region
    s_bytes = 16 if args.prec == "fp64" else 8
    pair_bytes = nr * s_bytes
    cap = int(os.environ.get("FX_WORK_MB", "2048")) << 20
    nk = min(Nt, max(1, cap // pair_bytes))
    nj = min(N, max(1, (cap // pair_bytes) // nk))
    if os.environ.get("FX_VX_NJ"):
        nj = min(nj, int(os.environ["FX_VX_NJ"]))
    multi = nj < N
    kern = {}
    for name in ("vx_plane_fwd", "vx_pencil_z", "vx_plane_inv", "convert"):
        cnt, ms = ctx.prof_read(fock.KERNEL_IDS[name])
        if cnt:
            kern[name] = {"launches": cnt, "avg_ms": ms / cnt, "total_ms": ms}
    ctx.prof_enable(False)
    dom = max((k for k in kern if k.startswith("vx_")), key=lambda k: kern[k]["total_ms"])
    pairs_per_launch = (nk * nj) if dom != "vx_plane_inv" else nk * nj
    bpp = algorithmic_bytes_per_pt(dom, s_bytes, nj, multi)
    bytes_per_launch = bpp * nr * pairs_per_launch
    achieved = bytes_per_launch / (kern[dom]["avg_ms"] * 1e-3) / 1e9
    traffic = None
    cpath = os.path.join(ROOT, "profiles", "vx_counters.json")
    if os.path.exists(cpath):
        c = json.load(open(cpath))
        if c.get("source_hash") == kernel_source_hash() and c.get("kernel") == dom and c.get("prec") == args.prec:
            traffic = c.get("bytes_per_launch")
    for k in kern:
        if k.startswith("vx_"):
            b = algorithmic_bytes_per_pt(k, s_bytes, nj, multi) * nr * nk * nj
            kern[k]["algorithmic_GBps"] = b / (kern[k]["avg_ms"] * 1e-3) / 1e9

    result = {
        "metric": "Fock-exchange orbital pairs/s",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: V_X apply, {n}^3 grid, L={L:.2f} bohr, {N} orbitals x {Nt} targets "
                         f"= {pairs} pair Poisson solves, HSE w=0.106"),
            "prec": args.prec,
            "accumulation": "f64" if args.prec in ("fp64", "fp32acc64") else "f32",
            "pairs_per_step": pairs,
            "batch": {"targets": nk, "orbitals": nj},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_pair_pt": bpp,
            "pairs_per_launch": pairs_per_launch,
        },
        "kernels": kern,
    }
    # model: whole-path algorithmic bytes / step time
    total_bpp = sum(algorithmic_bytes_per_pt(k, s_bytes, nj, multi)
                    for k in ("vx_plane_fwd", "vx_pencil_z", "vx_plane_inv"))
    result["path_model_GBps"] = total_bpp * nr * pairs / (ms_per_step * 1e-3) / 1e9

    if args.fp64_steps > 0 and args.prec != "fp64":
        del out
        P64 = P.to(torch.complex128)
        out64 = torch.empty((Nt, n, n, n), dtype=torch.complex128, device=dev)
        kw64 = dict(kw, prec="fp64", out=out64)
        ctx.apply_vx(P64, P64[:Nt], **kw64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            ctx.apply_vx(P64, P64[:Nt], **kw64)
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t0
        v64 = pairs * args.fp64_steps / el64
        result["fp64_same_gpu"] = {"value": v64, "unit": "pairs/s", "ms_per_step": 1e3 * el64 / args.fp64_steps,
                                   "speedup_of_value": value / v64}
        log(f"[bench] fp64 {v64:.0f} pairs/s")
        del P64, out64

    if args.cpu_seconds > 0:
        log("[bench] CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(psi_h, w, args.cpu_seconds)
    ctx.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
