"""Benchmark of the overlap-operator hot path on one MI355X.

Workload (default): 24^3 x 64 periodic lattice, links U = exp(i 0.25 H)
(seeded, synthetic), rho = 1.5, the 100 H_w eigenvectors closest to zero
projected, polynomial sign to delta = 1e-10, 12 spin x colour point sources
at the origin, quark masses 0.01 and 0.05, FP16 link and spinor storage with
FP32 arithmetic (FP64 projection inner products and reductions).

A timed step is the operator work of one CG iteration on the 12 sources:
one batched D(m) apply and one batched D(m)^dag apply (each: projection,
2n+1 stencil launches of the Clenshaw recursion, combine).  `value` is
overlap applies per second (each rhs counts once).  Also reported:
  dslash      - GB/s of the stencil (model bytes / HIP-event time) per
                precision and batch size, and the roofline of the dominant
                kernel (the FP16 12-real 12-rhs stencil);
  cg          - time to an FP64 true residual of 1e-10 for the mixed-
                precision 12-rhs solve (HIP-graph iterations) and for the
                plain FP64 solve, and their ratio;
  cpu_baseline- the FP64 numpy oracle on the host, on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cg]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dslash GB/s + D_ov applies/s at 24^3x64; CG time to 1e-10 vs plain FP64"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch from two rocprofv3 counter passes (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0, factors from a plain 1 GiB copy), keyed by the F16 12-rhs
# stencil configuration: (extra epilogue vectors, tuned shape kr, bs, pipe,
# rin, tm).  Summary and commands: profiles/stencil_f16_12rhs_24x24x24x64_counters.md
PROFILED_TRAFFIC = {
    (3, (2, 128, 0, 0, 0)): 4080216064,
    (0, (2, 128, 0, 0, 0)): 3094016000,
    (3, (2, 256, 0, 0, 0)): 4072608000,
    (0, (2, 256, 0, 0, 0)): 3037061120,
    (3, (2, 128, 0, 0, 4)): 3638409216,
    (0, (2, 128, 0, 0, 4)): 2811045888,
    (3, (2, 128, 0, 0, 8)): 3599534080,
    (0, (2, 128, 0, 0, 8)): 2698047488,
    (3, (2, 256, 0, 0, 4)): 3534860288,
    (0, (2, 256, 0, 0, 4)): 2486437888,
    (3, (2, 256, 0, 0, 8)): 3578030699,
    (0, (2, 256, 0, 0, 8)): 2634959975,
}


LAST_EIG = {}  # statistics of the latest spectral set-up's eigensolver


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=str, default="24,24,24,64")
    ap.add_argument("--ell", type=int, default=100)
    ap.add_argument("--delta", type=float, default=1e-10)
    ap.add_argument("--prec", type=str, default="f16")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--cg-masses", type=str, default="0.01,0.05")
    ap.add_argument("--inner-delta", type=float, default=1e-3,
                    help="sign accuracy of the inner (low-precision) operator; 0 = same as outer")
    ap.add_argument("--inner-tol", type=float, default=1e-3)
    ap.add_argument("--graph-chunk", type=int, default=8)
    ap.add_argument("--fp64-cg-rhs", type=int, default=1,
                    help="rhs of the full plain FP64 CG solve (its iteration count and time, scaled to 12); 0 = skip")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", choices=["full", "kernels", "learned"], default="full",
                    help="kernels: only a 1 GiB calibration copy and the stencil configurations "
                         "(for rocprofv3 counter passes); learned: train the PTC preconditioner on "
                         "16^3x32 fields and compare FGCR(net), FGCR(M=1) and CG on the --dims field")
    ap.add_argument("--pairs", type=int, default=2000, help="learned mode: training pairs (four fields)")
    ap.add_argument("--restart", type=int, default=16, help="learned mode: FGCR restart length")
    ap.add_argument("--cpu-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-data", type=str, default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-seed", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--no-c2", action="store_true", help="skip the 16^3x32 block (C2)")
    ap.add_argument("--rational-n", type=int, default=18,
                    help="order of the rational sign compared with the polynomial (0 skips the comparison)")
    ap.add_argument("--deflate", type=int, default=0,
                    help="chiral-sector eigenvectors for a deflated 12-rhs CG at the main workload (0 = skip)")
    ap.add_argument("--deflate-eig", type=str, default="f32:1e-7:1e-5",
                    help="with --deflate: comma-separated prec:sign_delta:tol of the overlap eigensolver runs")
    ap.add_argument("--deflate-mr", action="store_true",
                    help="with --deflate: also solve with the minimal-residual form of the same deflation")
    ap.add_argument("--defl-ell", type=int, default=16,
                    help="16^3x32 block: chiral-sector eigenvectors for the deflated CG (eq. 9); 0 skips it")
    ap.add_argument("--shape", type=str, default="",
                    help="kernels mode: pin the 12-rhs stencil shape kr,bs,pipe,rin,tm for the sign applications")
    ap.add_argument("--fp64-batched-iters", type=int, default=12,
                    help="inner iterations timed for the batched 12-rhs plain FP64 CG (0 = skip)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, timed in a child process limited to one thread
# ---------------------------------------------------------------------------
def cpu_baseline_child(dims, n, ell, data_dir, seed):
    """One single-threaded oracle process: 3 H_w applications and the
    projection on 4 vectors, on the links in data_dir (written once by the
    parent) and a spinor of its own seed."""
    import numpy as np

    import synth_inputs as si
    from oracle import dirac, sign
    from oracle.lattice import Lattice

    lat = Lattice(dims)
    U = np.load(os.path.join(data_dir, "links.npy"), mmap_mode="r")
    U = np.ascontiguousarray(U)
    psi = si.gaussian_spinor(dims, 103 + seed)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        dirac.hw_apply(lat, U, psi, 1.5)
    t_dw = (time.perf_counter() - t0) / reps
    # projection on ell vectors: time it on 4 vectors and scale linearly
    V = np.stack([si.gaussian_spinor(dims, 200 + i) for i in range(4)])
    t0 = time.perf_counter()
    sign.project_low(V, psi)
    t_proj4 = time.perf_counter() - t0
    t_apply = t_dw * (2 * n + 1) + t_proj4 * ell / 4.0
    print(json.dumps({"t_dw": t_dw, "t_proj4": t_proj4, "t_apply": t_apply, "reps": reps}))


def _cpu_children(dims, n, ell, data_dir, nproc):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    env["HIP_VISIBLE_DEVICES"] = ""
    procs = []
    for k in range(nproc):
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-only", "--dims", ",".join(map(str, dims)),
               "--ell", str(ell), "--delta", str(n), "--cpu-data", data_dir, "--cpu-seed", str(k)]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env))
    out = []
    for pr in procs:
        so, se = pr.communicate(timeout=900)
        if pr.returncode != 0:
            raise RuntimeError("cpu baseline child failed: " + se[-2000:])
        out.append(json.loads(so.strip().splitlines()[-1]))
    return out


def cpu_model():
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        for line in txt.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(dims, n, ell, data_dir):
    """The oracle on this host: one process alone (1 thread), then one
    single-threaded process per core of the job's CPU share at once (numpy's
    stencil is single-threaded, so processes are how it uses every core).
    Throughput = sum over processes of 1 / (time of one extrapolated apply)."""
    nproc_host = os.cpu_count() or 1
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    cores = max(1, min(nproc_host, share if share > 0 else nproc_host, 16))
    one = _cpu_children(dims, n, ell, data_dir, 1)[0]
    many = _cpu_children(dims, n, ell, data_dir, cores) if cores > 1 else [one]
    v1 = 1.0 / one["t_apply"]
    vall = sum(1.0 / d["t_apply"] for d in many)
    t_dw_all = sum(d["t_dw"] for d in many) / len(many)
    return {
        "value": vall,
        "unit": "D_ov applies/s",
        "cores": cores,
        "kind": "oracle",
        "sample": ("FP64 numpy oracle, %d single-threaded processes at once (one per core): each times 3 H_w "
                   "applications at %s (%.2f s each on average) and the projection on 4 vectors, extrapolated to "
                   "one overlap apply of 2n+1 = %d stencil applications and %d projected vectors; the same sample "
                   "alone on one thread: %.5f applies/s (H_w %.2f s)"
                   % (cores, "x".join(map(str, dims)), t_dw_all, 2 * n + 1, ell, v1, one["t_dw"])),
        "one_thread_value": v1,
        "nproc": nproc_host,
        "cpu_model": cpu_model(),
        "gflops_per_core_dslash": round(1368.0 * math.prod(dims) / one["t_dw"] / 1e9, 3),
    }


# ---------------------------------------------------------------------------
# Counter runs: a plain copy of known size, then each stencil configuration
# ---------------------------------------------------------------------------
def kernels_mode(dims, prec_name, shape=None):
    import numpy as np
    import torch

    import synth_inputs as si
    from paper_1106_4964_amd import ovl

    dev = torch.device("cuda:0")
    prec = ovl.PREC[prec_name]
    g = ovl.Geometry(dims)
    U = si.gauge_field(dims, 0.25, 3)
    gauge = ovl.Gauge(g, torch.from_numpy(U).to(dev))
    del U
    gauge.set_repr(prec, 1)
    gauge.set_repr(ovl.OVL_F32, 1)
    src = torch.from_numpy(np.stack([si.gaussian_spinor(dims, 500 + r) for r in range(12)])).to(dev)
    b64 = torch.empty(g.spinor_bytes(ovl.OVL_F64, 12), dtype=torch.uint8, device=dev)
    ovl.ovl_pack_spinor(g, src, b64, ovl.OVL_F64, 12, None)
    del src
    # calibration: copy 1 GiB (reads 1 GiB, writes 1 GiB)
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    log("calibration copy: %d bytes read and written per launch" % (a.numel() * 4))
    del a, c
    if shape:
        for nv in range(4):
            ovl.stencil_set_shape(g, prec, 1, nv, 12, shape)
    for name, p, nrhs in [("f16_12_12rhs", prec, 12), ("f16_12_1rhs", prec, 1),
                          ("f32_12_1rhs", ovl.OVL_F32, 1), ("f64_18_1rhs", ovl.OVL_F64, 1)]:
        x = torch.empty(g.spinor_bytes(p, nrhs), dtype=torch.uint8, device=dev)
        ovl.ovl_convert(g, b64[: g.spinor_bytes(ovl.OVL_F64, nrhs)], ovl.OVL_F64, x, p, nrhs, None)
        y = torch.empty_like(x)
        ovl.ovl_hw_apply(y, x, gauge, 1.5, p, nrhs, None)  # tunes the shape
        torch.cuda.synchronize()
        for _ in range(3):
            ovl.ovl_hw_apply(y, x, gauge, 1.5, p, nrhs, None)
        torch.cuda.synchronize()
        log("stencil %s: shape (kr, bs, pipe, rin, tm) = %s" % (name, ovl.stencil_shape(g, p, p != ovl.OVL_F64, 0, nrhs)))
    # the Clenshaw recurrence of the sign function on 12 rhs: its steps are
    # the stencil with 0 and with 3 extra epilogue vectors (in a pinned shape
    # when one is given, else the tuned one)
    x = torch.empty(g.spinor_bytes(prec, 12), dtype=torch.uint8, device=dev)
    ovl.ovl_convert(g, b64, ovl.OVL_F64, x, prec, 12, None)
    y = torch.empty_like(x)
    sgn = ovl.Sign(0.1, 6.4, n=6)
    for _ in range(6):  # the first call tunes; the last five run the tuned shapes
        ovl.ovl_sign_apply(y, x, gauge, 1.5, sgn, None, prec, 12, None)
    torch.cuda.synchronize()
    for nv in (0, 3):
        log("clenshaw stencil %s 12 rhs, %d extra vectors: shape (kr, bs, pipe, rin, tm) = %s"
            % (prec_name, nv, ovl.stencil_shape(g, prec, 1, nv, 12)))


# ---------------------------------------------------------------------------
def spectral_setup(ovl, g, gauge, dims, rho, ell, delta, seed_base, tol=1e-12):
    """Lanczos bound on |H_w|, the ell lowest |lambda| eigenpairs of H_w and
    the sign function for sqrt(eps) = |lambda_ell| / lambda_max."""
    import numpy as np
    import torch

    import synth_inputs as si

    dev = torch.device("cuda:0")
    log("Lanczos bound")
    v0 = torch.empty(g.spinor_bytes(ovl.OVL_F64), dtype=torch.uint8, device=dev)
    ovl.ovl_pack_spinor(g, torch.from_numpy(si.gaussian_spinor(dims, 17)[None]).to(dev), v0, ovl.OVL_F64, 1, None)
    lam = ctypes.c_double()
    ovl.ovl_hw_bound(gauge, rho, v0, 60, ctypes.byref(lam), None, None, None)
    lam_max = lam.value * (1 + 1e-6)
    del v0
    m = ell + max(12, ell // 4)
    log("eigensolver: %d of %d vectors" % (ell, m))
    # Gaussian start block drawn on the device (seeded): any full-rank start
    # serves the eigensolver, and host generation would take ~0.2 s a vector
    V = torch.empty(g.spinor_bytes(ovl.OVL_F64, m), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed_base)
    V.view(torch.float64).normal_(generator=gen)
    lams = np.zeros(ell)
    est = ovl.EigStats()
    rc = ovl.ovl_hw_eigs(gauge, rho, ell, m, V, lams, lam_max, tol, 60, 40, ctypes.byref(est), None)
    log("eigensolver rc %d: %d passes, %d H_w applies, max residual %.2e, %.1f s, |lambda_l| = %.4f"
        % (rc, est.iterations, est.hw_applies, est.max_residual, est.seconds, abs(lams[-1])))
    LAST_EIG.update(degree=40, passes=est.iterations, hw_applies=est.hw_applies, seconds=round(est.seconds, 2),
                    max_residual=est.max_residual)
    Vk = V[: ell * g.spinor_bytes(ovl.OVL_F64)]
    lm = ovl.LowModes(g, Vk, lams)
    sgn = ovl.Sign(abs(lams[-1]), lam_max, delta=delta)
    log("sign: n = %d, sqrt(eps) = %.4f, delta = %.2e" % (sgn.n, math.sqrt(sgn.eps), sgn.delta))
    return lam_max, lams, V, lm, sgn


# ---------------------------------------------------------------------------
def learned_mode(args, dims):
    """The learned preconditioner at scale: a 1-4-1 PTC network trained on
    (b, x) pairs harvested from plain CG solves on four 16^3x32 fields, then
    the right preconditioner of the batched FGCR for D(m) on the 24^3x64
    field, against mixed CG and FGCR with M = 1."""
    import numpy as np
    import torch

    import synth_inputs as si
    from paper_1106_4964_amd import ovl

    dev = torch.device("cuda:0")
    rho, mass, R = 1.5, 0.01, 12
    prec = ovl.PREC[args.prec]
    F32, F64 = ovl.OVL_F32, ovl.OVL_F64
    tdims = (16, 16, 16, 32)
    pairs_per_field = args.pairs // 4
    tg = ovl.Geometry(tdims)
    vb = tg.spinor_bytes(F32)
    fields = []
    t0 = time.perf_counter()
    harvest = []
    for seed in (41, 42, 43, 44):
        log("training field %s seed %d" % (tdims, seed))
        gt = ovl.Gauge(tg, torch.from_numpy(si.gauge_field(tdims, 0.25, seed)).to(dev))
        gt.set_repr(F32, 0)
        _, lams_t, Vt, lmt, st_ = spectral_setup(ovl, tg, gt, tdims, rho, 20, 1e-8, 100 * seed, tol=1e-10)
        sin_t = ovl.Sign(abs(lams_t[-1]), st_.lam_max, delta=args.inner_delta)
        # (b, x) pairs from plain CG: the FP32 search directions p of the
        # inner iterations and their images b = D(m) p, every 8th iteration,
        # from batches of 12 Gaussian sources until the buffers are full
        X = torch.empty(tg.spinor_bytes(F32, pairs_per_field), dtype=torch.uint8, device=dev)
        B = torch.empty_like(X)
        got, batch, cg_its = 0, 0, 0
        while got < pairs_per_field:
            blk = np.stack([si.gaussian_spinor(tdims, 10000 * seed + 12 * batch + j) for j in range(12)])
            b64t = torch.empty(tg.spinor_bytes(F64, 12), dtype=torch.uint8, device=dev)
            ovl.ovl_pack_spinor(tg, torch.from_numpy(blk).to(dev), b64t, F64, 12, None)
            xt = torch.zeros_like(b64t)
            opts = ovl.SolveOpts(F32, 1e-5, 0, 1, 60, X[got * vb:].data_ptr(), B[got * vb:].data_ptr(),
                                 pairs_per_field - got, sin_t.handle.value)
            opts.harvest_stride = 8
            stt = ovl.SolveStats()
            ovl.ovl_cg_solve(xt, b64t, 12, gt, rho, mass, st_, lmt, 1e-8, 20000, opts, ctypes.byref(stt), None)
            got += stt.harvested
            cg_its += stt.iterations
            batch += 1
        torch.cuda.synchronize()
        harvest.append({"seed": seed, "pairs": got, "cg_batches": batch, "cg_iterations": cg_its})
        log("harvested %d pairs from %d CG solves of 12 sources (%d iterations)" % (got, batch, cg_its))
        fields.append((gt, X, B, Vt, lmt, st_))
    t_pairs = time.perf_counter() - t0
    net_t = ovl.Net(tg, 4)
    rng = np.random.default_rng(5)
    w1 = 0.02 * (rng.standard_normal((9, 4, 1, 4, 4)) + 1j * rng.standard_normal((9, 4, 1, 4, 4)))
    w2 = 0.02 * (rng.standard_normal((9, 1, 4, 4, 4)) + 1j * rng.standard_normal((9, 1, 4, 4, 4)))
    w1[0, 0, 0] += np.eye(4)
    w2[0, 0, 0] += np.eye(4) / rho
    net_t.set_weights(w1, w2)
    losses = []
    t0 = time.perf_counter()
    for rnd, (epochs, lr) in enumerate([(3, 1e-3), (2, 3e-4)]):
        for (gt, X, B, _, _, _) in fields:
            order = np.concatenate([rng.permutation(pairs_per_field) for _ in range(epochs)]).astype(np.int32)
            hist = np.zeros(epochs)
            ovl.ovl_net_train(net_t, gt, B, X, pairs_per_field, epochs, 8, lr, order, hist, None)
            losses.append([round(float(v), 5) for v in hist])
            log("training round %d: loss %s" % (rnd, losses[-1]))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w1t, w2t = net_t.get_weights()
    del fields, net_t

    log("test field %s" % (dims,))
    g = ovl.Geometry(dims)
    gauge = ovl.Gauge(g, torch.from_numpy(si.gauge_field(dims, 0.25, 3)).to(dev))
    gauge.set_repr(prec, 1)
    gauge.set_repr(F32, 0)
    gauge.set_repr(F32, 1)
    lam_max, lams, V, lm, sgn = spectral_setup(ovl, g, gauge, dims, rho, args.ell, args.delta, 1000)
    sgn_in = ovl.Sign(abs(lams[-1]), lam_max, delta=args.inner_delta)
    net = ovl.Net(g, 4)
    net.set_weights(w1t, w2t)
    b64 = torch.empty(g.spinor_bytes(F64, R), dtype=torch.uint8, device=dev)
    ovl.ovl_pack_spinor(g, torch.from_numpy(si.point_sources(dims)).to(dev), b64, F64, R, None)
    out = {}
    for name, M in [("cg", None), ("fgcr_net", net), ("fgcr_identity", None)]:
        x = torch.zeros(g.spinor_bytes(F64, R), dtype=torch.uint8, device=dev)
        opts = ovl.SolveOpts(prec, args.inner_tol, args.graph_chunk if name == "cg" else 0, 1, 60, None, None, 0,
                             sgn_in.handle.value)
        st = ovl.SolveStats()
        if name == "cg":
            rc = ovl.ovl_cg_solve(x, b64, R, gauge, rho, mass, sgn, lm, 1e-10, 20000, opts, st, None)
        else:
            rc = ovl.ovl_fgcr_solve(x, b64, R, gauge, rho, mass, sgn, lm, M, args.restart, 1e-10, 20000, opts, st,
                                    None)
        out[name] = {"rc": rc, "seconds": round(st.seconds, 2), "iterations": st.iterations,
                     "sign_applies": st.sign_applies, "fallback_used": st.fallback_used,
                     "max_true_residual": max(st.true_residual[r] for r in range(R))}
        log("%s: %s" % (name, out[name]))
    res = {
        "metric": "learned preconditioner: FGCR(net) vs CG and FGCR(M=1), time to 1e-10 at %s" % "x".join(map(str, dims)),
        "value": round(out["cg"]["seconds"] / out["fgcr_net"]["seconds"], 3),
        "unit": "speedup of FGCR(net) over mixed CG",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "12 point sources, m=%g, %s storage inner, %d low modes, delta %g (inner %g), "
                               "FGCR restart %d; net 1-4-1 trained on %d pairs from four %s fields"
                               % (mass, args.prec, args.ell, args.delta, args.inner_delta, args.restart, args.pairs,
                                  "x".join(map(str, tdims)))},
        "training": {"seconds_pairs": round(t_pairs, 1), "seconds_train": round(t_train, 1), "loss": losses,
                     "harvest": harvest},
        "solves": out,
    }
    print(json.dumps(res), flush=True)


# ---------------------------------------------------------------------------
def c2_block(ovl, args):
    """16^3x32 (the second workload): 50 projected H_w modes, sign to 1e-10;
    FP64 / FP32 / F16 storage: stencil GB/s and D(m) applies/s on one vector,
    and CG at m = 0.01 on one point source to an FP64 true residual of 1e-10
    (plain FP64, and mixed with an FP32 or F16 inner solve)."""
    import numpy as np
    import torch

    import synth_inputs as si

    dev = torch.device("cuda:0")
    dims, rho, m, ell = (16, 16, 16, 32), 1.5, 0.01, 50
    g = ovl.Geometry(dims)
    gauge = ovl.Gauge(g, torch.from_numpy(si.gauge_field(dims, 0.25, 2)).to(dev))
    for p in (ovl.OVL_F32, ovl.OVL_F16):
        gauge.set_repr(p, 1)
    t0 = time.perf_counter()
    lam_max, lams, V, lm, sgn = spectral_setup(ovl, g, gauge, dims, rho, ell, 1e-10, 2000)
    t_setup = time.perf_counter() - t0
    setup_eig = dict(LAST_EIG)
    sgn_in = ovl.Sign(abs(lams[-1]), lam_max, delta=1e-3)
    b64 = torch.empty(g.spinor_bytes(ovl.OVL_F64), dtype=torch.uint8, device=dev)
    ovl.ovl_pack_spinor(g, torch.from_numpy(si.point_source(dims, 0, 0)[None]).to(dev), b64, ovl.OVL_F64, 1, None)
    out = {"workload": "16x16x16x32, %d projected modes, sign delta 1e-10 (n=%d, sqrt(eps)=%.4f), m=%g, one point "
                       "source" % (ell, sgn.n, math.sqrt(sgn.eps), m),
           "setup_seconds": round(t_setup, 1)}
    N = g.N
    for name, p, L in [("f64", ovl.OVL_F64, 18), ("f32", ovl.OVL_F32, 12), ("f16", ovl.OVL_F16, 12)]:
        x = torch.empty(g.spinor_bytes(p), dtype=torch.uint8, device=dev)
        ovl.ovl_convert(g, b64, ovl.OVL_F64, x, p, 1, None)
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        bpr = {ovl.OVL_F64: 8, ovl.OVL_F32: 4, ovl.OVL_F16: 2}[p]
        t_dw = _event_time(lambda: ovl.ovl_hw_apply(y, x, gauge, rho, p, 1, None), 20)
        t_ov = _event_time(lambda: ovl.ovl_overlap_apply(z, x, gauge, rho, m, sgn, lm, 0, p, 1, None), 3)
        rec = {"dslash_us": round(t_dw * 1e6, 2), "dslash_model_GBps": round(N * bpr * (4 * L + 48) / t_dw / 1e9, 1),
               "overlap_applies_per_s": round(1.0 / t_ov, 2)}
        xs = torch.zeros(g.spinor_bytes(ovl.OVL_F64), dtype=torch.uint8, device=dev)
        if p == ovl.OVL_F64:
            opts = ovl.SolveOpts(p, 0.0, 0, 1, 60)
        else:
            opts = ovl.SolveOpts(p, 1e-3, 8, 1, 60, None, None, 0, sgn_in.handle.value)
        st = ovl.SolveStats()
        rc = ovl.ovl_cg_solve(xs, b64, 1, gauge, rho, m, sgn, lm, 1e-10, 20000, opts, st, None)
        rec["cg"] = {"rc": rc, "seconds": round(st.seconds, 3), "iterations": st.iterations, "restarts": st.restarts,
                     "true_residual": st.true_residual[0], "sign_applies": st.sign_applies,
                     "dslash_applies": st.dslash_applies}
        log("C2 %s: %s" % (name, rec))
        out[name] = rec
    out["cg_speedup_f16_vs_f64"] = round(out["f64"]["cg"]["seconds"] / out["f16"]["cg"]["seconds"], 2)
    out["cg_speedup_f32_vs_f64"] = round(out["f64"]["cg"]["seconds"] / out["f32"]["cg"]["seconds"], 2)
    # the paper's eigensolver filter degree (a Chebyshev polynomial T_100 of
    # H_w^2) against the default degree 40 of the set-up above
    m_basis = ell + max(12, ell // 4)
    Vt = torch.empty(g.spinor_bytes(ovl.OVL_F64, m_basis), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(2000)
    Vt.view(torch.float64).normal_(generator=gen)
    lt = np.zeros(ell)
    est = ovl.EigStats()
    rc = ovl.ovl_hw_eigs(gauge, rho, ell, m_basis, Vt, lt, lam_max, 1e-12, 60, 100, ctypes.byref(est), None)
    out["eigensolver_T100"] = {"rc": rc, "degree": 100, "passes": est.iterations, "hw_applies": est.hw_applies,
                               "seconds": round(est.seconds, 2), "max_residual": est.max_residual,
                               "max_abs_eigenvalue_diff_vs_degree40": float(np.max(np.abs(np.abs(lt) - np.abs(lams)))),
                               "degree40": setup_eig}
    log("C2 eigensolver with T_100: %s" % out["eigensolver_T100"])
    del Vt
    # adaptive precision (Sec. V): the same F16-inner solve with coarser
    # inner signs allowed in the cycles that need less than inner_tol
    relax = [ovl.Sign(abs(lams[-1]), lam_max, delta=d) for d in (1e-2, 1e-1)]
    arr = (ctypes.c_void_p * 2)(*[r.handle.value for r in relax])
    opts = ovl.SolveOpts(ovl.OVL_F16, 1e-3, 8, 1, 60, None, None, 0, sgn_in.handle.value)
    opts.relax_signs = ctypes.cast(arr, ctypes.c_void_p).value
    opts.n_relax = 2
    xs = torch.zeros(g.spinor_bytes(ovl.OVL_F64), dtype=torch.uint8, device=dev)
    st = ovl.SolveStats()
    rc = ovl.ovl_cg_solve(xs, b64, 1, gauge, rho, m, sgn, lm, 1e-10, 20000, opts, st, None)
    base = out["f16"]["cg"]
    out["adaptive_sign_f16"] = {"rc": rc, "seconds": round(st.seconds, 3), "iterations": st.iterations,
                                "restarts": st.restarts, "sign_applies": st.sign_applies,
                                "dslash_applies": st.dslash_applies, "true_residual": st.true_residual[0],
                                "fixed_inner_sign": {"n": sgn_in.n, "seconds": base["seconds"],
                                                     "sign_applies": base["sign_applies"],
                                                     "dslash_applies": base["dslash_applies"]},
                                "relax_signs_n": [r.n for r in relax]}
    log("C2 adaptive inner sign: %s" % out["adaptive_sign_f16"])
    if args.defl_ell > 0:
        out["deflation"] = deflation_block(ovl, g, gauge, rho, m, sgn, sgn_in, lm, b64, args.defl_ell, out)
    del lm, V
    return out


def deflation_block(ovl, g, gauge, rho, m, sgn, sgn_in, lm, b64, ell, plain):
    """Eigenpairs of D closest to zero from ell eigenvectors of one chiral
    sector (FP64 sign with the projected modes), then the same CG solves as
    above with eq. 9 deflation, reported beside the undeflated ones."""
    import ctypes

    import numpy as np
    import torch

    import synth_inputs as si

    dev = torch.device("cuda:0")
    V = torch.empty(g.spinor_bytes(ovl.OVL_F64, 2 * ell), dtype=torch.uint8, device=dev)
    ovl.ovl_pack_spinor(g, torch.from_numpy(si.gaussian_spinor(g.dims, 7)[None]).to(dev), V, ovl.OVL_F64, 1, None)
    d = np.zeros(4 * ell)
    nout = ctypes.c_int()
    est = ovl.EigStats()
    K = min(512, max(2 * ell + 16, ell + 48))
    rc = ovl.ovl_overlap_eigs(gauge, rho, sgn, lm, ovl.OVL_F64, +1, ell, K, V, d, ctypes.byref(nout), 1e-9, 40,
                              ctypes.byref(est),
                              None)
    dc = d[: 2 * nout.value].view(np.complex128)
    rec = {"sector_vectors": ell, "lanczos_basis": K, "pairs_of_D": nout.value, "rc": rc,
           "eig_seconds": round(est.seconds, 2), "eig_restart_cycles": est.iterations,
           "eig_dslash_applies": est.hw_applies, "eig_max_residual": est.max_residual,
           "abs_d_min": float(np.abs(dc[0])), "abs_d_max": float(np.abs(dc[-1]))}
    defl = ovl.Deflation(g, V, dc)
    for name, p in (("f64", ovl.OVL_F64), ("f16", ovl.OVL_F16)):
        xs = torch.zeros(g.spinor_bytes(ovl.OVL_F64), dtype=torch.uint8, device=dev)
        if p == ovl.OVL_F64:
            opts = ovl.SolveOpts(p, 0.0, 0, 1, 60)
        else:
            opts = ovl.SolveOpts(p, 1e-3, 8, 1, 60, None, None, 0, sgn_in.handle.value)
        opts.deflation = defl.handle.value
        st = ovl.SolveStats()
        rc = ovl.ovl_cg_solve(xs, b64, 1, gauge, rho, m, sgn, lm, 1e-10, 20000, opts, st, None)
        base = plain[name]["cg"]
        rec["cg_" + name] = {"rc": rc, "seconds": round(st.seconds, 3), "iterations": st.iterations,
                             "restarts": st.restarts, "true_residual": st.true_residual[0],
                             "undeflated_iterations": base["iterations"], "undeflated_seconds": base["seconds"],
                             "iteration_ratio": round(st.iterations / max(1, base["iterations"]), 3)}
    log("C2 deflation: %s" % rec)
    del defl, V
    return rec


def sign_comparison(ovl, g, gauge, rho, lams, lam_max, V, lm, sgn, args):
    """The paper's comparison of sign approximations (Sec. V): one FP64
    sign(H_w) application on a Gaussian vector with the same projected low
    modes, by the polynomial (Clenshaw) and by the rational function of order
    rational_n (multi-shift CG and double pass, Krylov tolerance 1e-10);
    time, H_w applications and the difference between the results."""
    import numpy as np
    import torch

    import synth_inputs as si

    dev = torch.device("cuda:0")
    v64 = g.spinor_bytes(ovl.OVL_F64)
    psi = torch.empty(v64, dtype=torch.uint8, device=dev)
    ovl.ovl_pack_spinor(g, torch.from_numpy(si.gaussian_spinor(g.dims, 77)[None]).to(dev), psi, ovl.OVL_F64, 1, None)
    ref = torch.empty_like(psi)
    t_poly = _event_time(lambda: ovl.ovl_sign_apply(ref, psi, gauge, rho, sgn, lm, ovl.OVL_F64, 1, None), 3)
    rat = ovl.Rational(abs(lams[-1]), lam_max, args.rational_n)
    out = {"workload": "one FP64 vector, %s lattice, %d projected modes" % ("x".join(map(str, g.dims)), len(lams)),
           "polynomial": {"n": sgn.n, "delta": sgn.delta, "seconds": round(t_poly, 4), "hw_applies": 2 * sgn.n + 1},
           "rational_n": rat.n, "rational_delta": rat.delta}
    pn = torch.linalg.vector_norm(ref.view(torch.float64)).item()
    for name, method in (("multishift_cg", 0), ("double_pass", 1)):
        res = torch.empty_like(psi)
        st = ovl.RationalStats()
        rc = ovl.ovl_rational_sign_apply(res, psi, gauge, rho, rat, lm, method, 1e-10, 5000, ctypes.byref(st), None)
        diff = torch.linalg.vector_norm(res.view(torch.float64) - ref.view(torch.float64)).item() / pn
        out[name] = {"rc": rc, "seconds": round(st.seconds, 4), "krylov_steps": st.iterations,
                     "hw_applies": st.hw_applies, "rel_diff_vs_polynomial": diff,
                     "time_vs_polynomial": round(st.seconds / t_poly, 2)}
        log("sign comparison %s: %s" % (name, out[name]))
    return out


def _event_time(fn, reps):
    """Seconds per call of fn, timed with HIP events on torch's current stream
    (the stream the library's kernels are launched on) after one warm-up."""
    import torch

    fn()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def _event_time_cold(fn, reps, scratch):
    """Median seconds of single calls of fn, each after writing a 1 GiB
    scratch buffer (evicts L2 and the 256 MB MALL), timed with HIP events."""
    import torch

    fn()
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        scratch.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    ts.sort()
    return ts[len(ts) // 2]


def main():
    args = parse()
    dims = tuple(int(v) for v in args.dims.split(","))
    if args.cpu_only:
        cpu_baseline_child(dims, int(args.delta), args.ell, args.cpu_data, args.cpu_seed)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the whole lattice lives in one MI355X's HBM and this build "
              "has no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.mode == "kernels":
        kernels_mode(dims, args.prec, tuple(int(v) for v in args.shape.split(",")) if args.shape else None)
        return
    if args.mode == "learned":
        os.environ.setdefault("OVL_LOG", "1")
        learned_mode(args, dims)
        return
    os.environ.setdefault("OVL_LOG", "1")  # solver progress lines on stderr
    import ctypes
    import tempfile

    import numpy as np
    import torch

    import synth_inputs as si
    from paper_1106_4964_amd import ovl

    dev = torch.device("cuda:0")
    rho = 1.5
    masses = tuple(float(v) for v in args.cg_masses.split(","))
    prec = ovl.PREC[args.prec]
    R = 12
    t_setup = time.perf_counter()

    log("gauge field %s" % (dims,))
    g = ovl.Geometry(dims)
    U = si.gauge_field(dims, 0.25, 3)
    gauge = ovl.Gauge(g, torch.from_numpy(U).to(dev))
    cpu_dir = None
    if not args.no_cpu:
        # the CPU baseline's processes read the same links from a file
        cpu_dir = tempfile.mkdtemp(prefix="ovl_bench_")
        np.save(os.path.join(cpu_dir, "links.npy"), U)
    del U
    gauge.set_repr(prec, 1)
    gauge.set_repr(ovl.OVL_F32, 1)

    def pack(a, p, n):
        out = torch.empty(g.spinor_bytes(p, n), dtype=torch.uint8, device=dev)
        ovl.ovl_pack_spinor(g, torch.from_numpy(np.ascontiguousarray(a)).to(dev), out, p, n, None)
        return out

    lam_max, lams, V, lm, sgn = spectral_setup(ovl, g, gauge, dims, rho, args.ell, args.delta, 1000)
    ell = args.ell

    b64 = pack(si.point_sources(dims), ovl.OVL_F64, R)
    bP = torch.empty(g.spinor_bytes(prec, R), dtype=torch.uint8, device=dev)
    ovl.ovl_convert(g, b64, ovl.OVL_F64, bP, prec, R, None)
    y1 = torch.empty_like(bP)
    y2 = torch.empty_like(bP)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    log("setup %.1f s" % t_setup)

    # ---------------------------------------------------------------- steps
    def step(p=prec, xin=bP, a=y1, b=y2):
        ovl.ovl_overlap_apply(a, xin, gauge, rho, masses[0], sgn, lm, 0, p, R, None)
        ovl.ovl_overlap_apply(b, a, gauge, rho, masses[0], sgn, lm, 1, p, R, None)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ovl.ovl_stencil_timer(1)  # HIP events around every stencil launch of the timed steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ovl.ovl_stencil_timer(0)
    step_kernels = {}
    for nv in range(4):
        n_l, ms_l = ovl.stencil_timer_read(prec, 1, nv, R)
        if n_l:
            step_kernels[nv] = (n_l, ms_l)
            log("timed steps: stencil %s-12 %d rhs, %d extra vectors: %d launches, avg %.1f us, %.1f%% of step time"
                % (args.prec, R, nv, n_l, 1e3 * ms_l / n_l, 100.0 * ms_l / (1e3 * t_steps)))
    ms_per_step = 1e3 * t_steps / args.steps
    applies_per_s = 2 * R * args.steps / t_steps
    log("step %.2f ms -> %.1f D_ov applies/s" % (ms_per_step, applies_per_s))

    # the same step with BF16 storage (two timed steps)
    gauge.set_repr(ovl.OVL_BF16, 1)
    bB = torch.empty(g.spinor_bytes(ovl.OVL_BF16, R), dtype=torch.uint8, device=dev)
    ovl.ovl_convert(g, b64, ovl.OVL_F64, bB, ovl.OVL_BF16, R, None)
    zB1, zB2 = torch.empty_like(bB), torch.empty_like(bB)
    step(ovl.OVL_BF16, bB, zB1, zB2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        step(ovl.OVL_BF16, bB, zB1, zB2)
    torch.cuda.synchronize()
    bf16_applies = 2 * R * 2 / (time.perf_counter() - t0)
    log("BF16 storage: %.1f D_ov applies/s" % bf16_applies)
    del bB, zB1, zB2

    # ------------------------------------------------------------- dslash
    N = g.N
    bytes_per_real = {ovl.OVL_F64: 8, ovl.OVL_F32: 4, ovl.OVL_F16: 2, ovl.OVL_BF16: 2}

    def model_bytes(p, L, nrhs, nv=0):
        # compulsory traffic, full lattice, one pass: links once per launch,
        # each input and output spinor once, each extra epilogue vector once
        return N * bytes_per_real[p] * (4 * L + 48 * nrhs + 24 * nv * nrhs)

    scratch = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
    dslash = {}
    gauge.set_repr(ovl.OVL_F64, 0)
    for p in (ovl.OVL_F32, ovl.OVL_F16, ovl.OVL_BF16):
        gauge.set_repr(p, 1)
    for name, p, L, nrhs in [("f64_18_1rhs", ovl.OVL_F64, 18, 1), ("f64_18_12rhs", ovl.OVL_F64, 18, 12),
                             ("f32_12_1rhs", ovl.OVL_F32, 12, 1), ("f32_12_12rhs", ovl.OVL_F32, 12, 12),
                             ("f16_12_1rhs", ovl.OVL_F16, 12, 1), ("f16_12_12rhs", ovl.OVL_F16, 12, 12),
                             ("bf16_12_1rhs", ovl.OVL_BF16, 12, 1), ("bf16_12_12rhs", ovl.OVL_BF16, 12, 12)]:
        x = torch.empty(g.spinor_bytes(p, nrhs), dtype=torch.uint8, device=dev)
        ovl.ovl_convert(g, b64[: g.spinor_bytes(ovl.OVL_F64, nrhs)], ovl.OVL_F64, x, p, nrhs, None)
        y = torch.empty_like(x)
        fn = lambda: ovl.ovl_hw_apply(y, x, gauge, rho, p, nrhs, None)  # noqa: E731
        t = _event_time(fn, 20)
        tc = _event_time_cold(fn, 20, scratch)
        mb = model_bytes(p, L, nrhs)
        dslash[name] = {"us": round(t * 1e6, 2), "model_GBps": round(mb / t / 1e9, 1),
                        "cold_us": round(tc * 1e6, 2), "cold_model_GBps": round(mb / tc / 1e9, 1),
                        "gflops": round(1368.0 * N * nrhs / t / 1e9, 1),
                        "shape": list(ovl.stencil_shape(g, p, p != ovl.OVL_F64, 0, nrhs))}
        log("dslash %s: warm %.1f us (%.0f GB/s), cold %.1f us (%.0f GB/s) (model bytes)"
            % (name, t * 1e6, mb / t / 1e9, tc * 1e6, mb / tc / 1e9))
        del x, y
    del scratch
    # dominant kernel of the timed steps: the stencil configuration with the
    # largest summed launch time, its average launch measured with HIP events
    dom_nv = max(step_kernels, key=lambda k: step_kernels[k][1])
    n_dom, ms_dom = step_kernels[dom_nv]
    dom_us = 1e3 * ms_dom / n_dom
    dom_bytes = model_bytes(prec, 12, R, dom_nv)
    dom_gbs = dom_bytes / (dom_us * 1e-6) / 1e9
    dom_shape = tuple(ovl.stencil_shape(g, prec, 1, dom_nv, R))
    profiled = dims == (24, 24, 24, 64) and R == 12 and args.prec == "f16"
    traffic = PROFILED_TRAFFIC.get((dom_nv, dom_shape)) if profiled else None
    roofline = {
        "bound": "hbm",
        "achieved": round(dom_gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "stencil_kernel<%s, 12-real links, %d extra vectors>, %d rhs, %s"
                  % (args.prec.upper(), dom_nv, R, "x".join(map(str, dims))),
        "bytes_per_launch": dom_bytes,
        "avg_launch_us": round(dom_us, 2),
        "launches": n_dom,
        "share_of_step": round(ms_dom / (1e3 * t_steps), 4),
        "shape": list(dom_shape),
    }

    # ----------------------------------------------------------------- CG
    cg = None
    if not args.no_cg:
        cg = {}

        sgn_in = None
        if args.inner_delta > 0:
            sgn_in = ovl.Sign(abs(lams[-1]), lam_max, delta=args.inner_delta)
            log("inner sign: n = %d (delta %.1e)" % (sgn_in.n, sgn_in.delta))
            cg["inner_sign_order"] = sgn_in.n

        def solve(p, nrhs, m, graph, inner_tol, inner_sign=None, maxiter=20000, deflation=None):
            x = torch.zeros(g.spinor_bytes(ovl.OVL_F64, nrhs), dtype=torch.uint8, device=dev)
            opts = ovl.SolveOpts(p, inner_tol, graph, 1, 60, None, None, 0,
                                 inner_sign.handle.value if inner_sign is not None else None)
            if deflation is not None:
                opts.deflation = deflation.handle.value
            st = ovl.SolveStats()
            rc = ovl.ovl_cg_solve(x, b64[: g.spinor_bytes(ovl.OVL_F64, nrhs)], nrhs, gauge, rho, m, sgn, lm,
                                  1e-10, maxiter, opts, st, None)
            res = max(st.true_residual[r] for r in range(nrhs))
            return {"rc": rc, "seconds": round(st.seconds, 3), "iterations": st.iterations,
                    "restarts": st.restarts, "max_true_residual": res, "sign_applies": st.sign_applies}

        for m in masses:
            r_mixed = solve(prec, R, m, args.graph_chunk, args.inner_tol, sgn_in)
            log("CG mixed m=%.2f: %s" % (m, r_mixed))
            cg["mixed_%s_12rhs_m%.2f" % (args.prec, m)] = r_mixed
        m0 = masses[0]
        if args.deflate > 0:
            # eq. 9 at this workload: 2 x deflate eigenpairs of D from one
            # chiral sector (the sector operator's sign at the given storage
            # precision and delta, with the projected modes), then the same
            # mixed 12-rhs solve with deflation in every FP64 cycle
            ellp = args.deflate
            base = cg["mixed_%s_12rhs_m%.2f" % (args.prec, m0)]
            for spec in args.deflate_eig.split(","):
                pname, sdelta, stol = spec.split(":")
                eprec, sdelta, stol = ovl.PREC[pname], float(sdelta), float(stol)
                sgn_eig = ovl.Sign(abs(lams[-1]), lam_max, delta=sdelta)
                Vd = torch.empty(g.spinor_bytes(ovl.OVL_F64, 2 * ellp), dtype=torch.uint8, device=dev)
                ovl.ovl_pack_spinor(g, torch.from_numpy(si.gaussian_spinor(dims, 7)[None]).to(dev), Vd, ovl.OVL_F64,
                                    1, None)
                dd = np.zeros(4 * ellp)
                nout = ctypes.c_int()
                est = ovl.EigStats()
                Kb = min(512, max(2 * ellp + 16, ellp + 48))
                erc = ovl.ovl_overlap_eigs(gauge, rho, sgn_eig, lm, eprec, +1, ellp, Kb, Vd, dd, ctypes.byref(nout),
                                           stol, 60, ctypes.byref(est), None)
                dc = dd[: 2 * nout.value].view(np.complex128)
                defl = ovl.Deflation(g, Vd, dc)
                r_defl = solve(prec, R, m0, args.graph_chunk, args.inner_tol, sgn_in, deflation=defl)
                mr = None
                if args.deflate_mr:
                    # the minimal-residual form on the same pairs: Z = D(0) Xi
                    # with the solve's FP64 operator, then the same solve
                    Zd = torch.empty(g.spinor_bytes(ovl.OVL_F64, nout.value), dtype=torch.uint8, device=dev)
                    torch.cuda.synchronize()
                    tz = time.perf_counter()
                    defl.prepare(gauge, rho, sgn, lm, Zd)
                    torch.cuda.synchronize()
                    tz = time.perf_counter() - tz
                    r_mr = solve(prec, R, m0, args.graph_chunk, args.inner_tol, sgn_in, deflation=defl)
                    mr = {"prepare_seconds": round(tz, 2), "cg": r_mr,
                          "iteration_ratio": round(r_mr["iterations"] / max(1, base["iterations"]), 3),
                          "eig_plus_prepare_plus_solve_vs_undeflated":
                              round((est.seconds + tz + r_mr["seconds"]) / base["seconds"], 3)}
                    del Zd
                rec = {"sector_vectors": ellp, "eig_prec": pname, "eig_sign_n": sgn_eig.n, "eig_sign_delta": sdelta,
                       "eig_tol": stol, "pairs_of_D": nout.value, "eig_rc": erc, "eig_seconds": round(est.seconds, 1),
                       "eig_restart_cycles": est.iterations, "eig_dslash_applies": est.hw_applies,
                       "eig_max_residual": est.max_residual, "abs_d_min": float(np.abs(dc[0])),
                       "abs_d_max": float(np.abs(dc[-1])), "cg": r_defl,
                       "iteration_ratio": round(r_defl["iterations"] / max(1, base["iterations"]), 3),
                       "time_ratio": round(r_defl["seconds"] / base["seconds"], 3),
                       "eig_plus_solve_vs_undeflated": round((est.seconds + r_defl["seconds"]) / base["seconds"], 3),
                       "minimal_residual": mr}
                cg["deflated_%s_12rhs_m%.2f_eig_%s" % (args.prec, m0, pname)] = rec
                log("CG deflated m=%.2f: %s" % (m0, rec))
                del defl, Vd
        if args.fp64_cg_rhs > 0:
            nfp = min(R, args.fp64_cg_rhs)
            r64 = solve(ovl.OVL_F64, nfp, m0, 0, 0.0)
            log("CG plain FP64 m=%.2f (%d rhs): %s" % (m0, nfp, r64))
            cg["plain_f64_m%.2f_%drhs" % (m0, nfp)] = r64
            t_sep = r64["seconds"] * (R / nfp)
            cg["plain_f64_12rhs_separate_seconds"] = round(t_sep, 2)
            if args.fp64_batched_iters > 0:
                # the 12 sources as one FP64 batch: the time per inner iteration
                # from two capped solves (k1 and k2 iterations; their fixed costs
                # - FP64 true residuals, first direction - cancel in the difference)
                k2 = max(2, args.fp64_batched_iters)
                k1 = max(1, k2 // 3)
                r1 = solve(ovl.OVL_F64, R, m0, 0, 0.0, maxiter=k1)
                r2 = solve(ovl.OVL_F64, R, m0, 0, 0.0, maxiter=k2)
                per_it = (r2["seconds"] - r1["seconds"]) / max(1, r2["iterations"] - r1["iterations"])
                t_bat = r2["seconds"] + per_it * max(0, r64["iterations"] - r2["iterations"])
                cg["plain_f64_12rhs_batched"] = {
                    "seconds_extrapolated": round(t_bat, 2), "seconds_per_iteration": round(per_it, 4),
                    "iterations_timed": [r1["iterations"], r2["iterations"]],
                    "iterations_assumed": r64["iterations"],
                    "note": ("the 12 point sources solved as one FP64 batch: time per inner iteration from solves "
                             "capped at %d and %d iterations, extended to the iteration count of the full FP64 "
                             "solve of one source (the 12 sources differ only in spin and colour)"
                             % (r1["iterations"], r2["iterations"]))}
                log("CG plain FP64 12 rhs batched: %.3f s per iteration -> %.1f s (extrapolated)" % (per_it, t_bat))
                t_den = t_bat
                cg["denominator"] = "plain FP64 CG on the 12 sources as one batch (extrapolated, see above)"
            else:
                t_den = t_sep
                cg["denominator"] = "plain FP64 CG, one source timed, times 12"
            key = "mixed_%s_12rhs_m%.2f" % (args.prec, m0)
            cg["speedup_vs_plain_f64_m%.2f" % m0] = round(t_den / cg[key]["seconds"], 2)
            cg["speedup_vs_plain_f64_separate_m%.2f" % m0] = round(t_sep / cg[key]["seconds"], 2)

    sign_cmp = None
    if args.rational_n > 0:
        log("sign comparison: polynomial vs rational (multi-shift CG, double pass)")
        sign_cmp = sign_comparison(ovl, g, gauge, rho, lams, lam_max, V, lm, sgn, args)

    c2 = None
    if not args.no_c2:
        log("C2 block (16x16x16x32)")
        c2 = c2_block(ovl, args)

    lib_live, lib_peak = ctypes.c_int64(), ctypes.c_int64()
    ovl.ovl_mem_stats(ctypes.byref(lib_live), ctypes.byref(lib_peak), 0)
    memory = {"library_peak_GB": round(lib_peak.value / 1e9, 2),
              "torch_peak_GB": round(torch.cuda.max_memory_allocated() / 1e9, 2),
              "note": "library: workspace pool, eigensolver basis and packed links; torch: fields and the "
                      "eigenvectors; the high-water mark is at most their sum"}
    log("device memory: %s" % memory)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        try:
            cpu = cpu_baseline(dims, sgn.n, ell, cpu_dir)
        finally:
            import shutil

            shutil.rmtree(cpu_dir, ignore_errors=True)
        log("cpu baseline: %s" % cpu)

    out = {
        "metric": METRIC,
        "value": round(applies_per_s, 3),
        "unit": "D_ov applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "overlap D(m) and D(m)^dag on 12 point sources, %s lattice, %s storage / f32 compute, "
                        "%d projected H_w modes, polynomial sign delta=%g (n=%d), m=%g"
                        % ("x".join(map(str, dims)), args.prec, ell, args.delta, sgn.n, masses[0]),
            "lattice": list(dims), "nrhs": R, "ell": ell, "sign_order": sgn.n,
            "sqrt_eps": round(math.sqrt(sgn.eps), 5), "lam_max": round(lam_max, 5), "rho": rho,
            "storage": args.prec, "links": "12-real", "setup_seconds": round(t_setup, 1),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "bf16_applies_per_s": round(bf16_applies, 3),
        "dslash": dslash,
        "cg": cg,
        "c2_16x16x16x32": c2,
        "sign_comparison": sign_cmp,
        "memory": memory,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
