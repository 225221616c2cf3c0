#!/usr/bin/env python
"""Benchmark of the QPAT Jacobian / priorconditioned-LSQR path on one MI355X.

Workload (default): 128^3 Kuhn voxels of a 40 mm cube (N = 2,146,689 nodes,
E = 12,582,912 tetrahedra), 16 Gaussian illuminations, seeded ellipsoid
phantom, linearised at the true phantom. A timed step is one J s + J^T t pair
(16 tangent and 16 adjoint solves as 16-RHS block PCG preconditioned by a
geometric-multigrid V-cycle, FP64, true residual <= 1e-10 ||b||). After the
timed pairs: seconds per priorconditioned-LSQR iteration (pair + M_delta^{-1}
+ reorthogonalisation), the same pair one right-hand side at a time and with
the Jacobi preconditioner (FP64 and mixed), live per-launch timing of the
PCG and V-cycle kernels for the roofline, and the FP64 CPU oracle timed on a
bounded sample of the same system.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "J·v+Jᵀ·w pairs/s & s per LSQR iter at 128³ grid; % HBM peak; plain vs batched"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(kind, N, layout, V, stat):
    """Bytes one launch must move, summed over the measured launches.

    Sliced ELL (any mesh): dir_spmv per active right-hand side reads r,
    p_old and writes p_new, q (4 N V), per launch the matrix (padded entries
    of V bytes + 4-byte columns, 4-byte row lengths) and the Jacobi diagonal
    (N V); update reads x, p, q, r and writes x, r (6 N V) + N V.
    Stencil form (lattice meshes): the direction kernel also applies the
    previous iteration's x += alpha p (read x, write x: 6 N V per right-hand
    side) and reads the operator as N (m+1) values; the update then reads q,
    r and writes r (3 N V) + N V.
    """
    L, lanes = stat["launches"], stat["lanes"]
    if layout["lattice"]:
        if kind == "dir_spmv":
            return lanes * 6 * N * V + L * (N * layout["stencil_arrays"] * V + N * V)
        return lanes * 3 * N * V + L * N * V
    if kind == "dir_spmv":
        op = layout["sell_len"] * (4 + V) + 4 * N
        return lanes * 4 * N * V + L * (op + N * V)
    return lanes * 6 * N * V + L * N * V


# the multigrid K kernels timed by the library (profile counters 4-7), the
# names rocprofv3 reports for them, and their algorithmic bytes: vectors of
# N B doubles per active right-hand side and the stencil rows (m + 1 doubles
# per node) and 1/a_ii once per launch
MG_KERNELS = {
    "K_mg_dir_spmv": ("k_mg_tile<0,16>", 3.5, True, False),  # read z (FP32), p_old; write p, q
    "K_mg_update": ("k_mgp_update<16>", 6, False, False),    # read x, p, r, q; write x, r
    "K_mg_resid0": ("k_mg_tile<1,16>", 2, True, True),       # read r; write r - A (w D^-1 r)
    "K_mg_smooth0": ("k_mg_tile<2,16>", 3, True, True),      # read x, r; write z
}
# on the tiled path counter 5 times the update fused with the finest-level
# residual (counter 6 then stays empty): read r, q; write r' and
# r' - A (w D^-1 r') in FP32 (half a vector); x is not touched there (the
# iterations keep their directions, and x is formed once per solve from them),
# and counter 7 the prolongation fused with the last sweep: read r, level 1's x
# (1/8 of the nodes, in FP32: 1/16 vector), the whole stencil rows (16 FP32
# values a node: the bytes of the stored form); write z in FP32 (half a vector)
MG_FUSED_UPDATE = ("k_mg_tile<6,16>", 3.5, 1, True)
MG_FUSED_SMOOTH = ("k_mg_prolong_smooth<false,true>", 1.5625, 1, True)


def mg_kernel(key, kst, p32=False):
    """(rocprofv3 name, vectors, stencil, 1/a_ii) of profile counter `key`; with
    p32 (mixed precision) the direction p is read and written in FP32: half a
    vector less in the direction kernel's read of the old p and its write of
    p."""
    fused = kst["K_mg_resid0"]["launches"] == 0
    if key == "K_mg_update" and fused:
        n, v, o, d = MG_FUSED_UPDATE
        return ("k_mg_tile<6,16,false,true>", v, o, d) if p32 else (n, v, o, d)
    if key == "K_mg_smooth0" and fused:   # mixed precision stages its x0 in FP32 (same HBM bytes)
        n, v, o, d = MG_FUSED_SMOOTH
        return ("k_mg_prolong_smooth<true,true>", v, o, d) if p32 else (n, v, o, d)
    n, v, o, d = MG_KERNELS[key]
    if p32 and key == "K_mg_dir_spmv":
        return ("k_mg_tile<0,16,true,true>", v - 1.0, o, d)
    return (n, v, o, d)


def mg_algorithmic_bytes(key, N, layout, stat, kst, p32=False):
    """Bytes one launch must move, summed over the measured launches."""
    _, vecs, op, diag = mg_kernel(key, kst, p32)
    per_launch = N * layout["stencil_arrays"] * 8 * int(op) + (N * 8 if diag else 0)
    return stat["lanes"] * vecs * N * 8 + stat["launches"] * per_launch


def mg_levels(nx, ny, nz, dense_max=1000, coarse_axis=5):
    """Node lattices of the K hierarchy: n -> n/2 + 1 per axis until the first
    coarse level of at most dense_max nodes (solved by its explicit inverse)."""
    lv = [(nx, ny, nz)]
    while max(lv[-1]) > coarse_axis and not (len(lv) >= 2 and np.prod(lv[-1]) <= dense_max):
        c = tuple(a // 2 + 1 if a > 2 else a for a in lv[-1])
        if c == lv[-1]:
            break
        lv.append(c)
    return [int(np.prod(v)) for v in lv]


def pair_algorithmic_bytes(N, E, levels, B, blocks, iters_tan, iters_adj, tiled27_min=16384, p32=False,
                           voxel=True):
    """Algorithmic HBM bytes of one J s + J^T t pair on the multigrid path: every
    kernel's reads and writes counted once (FP64 vectors of N B values; in
    FP32 the finest level's residual for the restriction, the V-cycle's output
    z and the last sweep's whole rows), with the measured PCG iteration counts.
    Per multigrid-PCG iteration (levels N_0 > N_1 > ...):
      finest level: direction + product 3.5 V_0 + rows, update + first residual
        3.5 V_0 + rows + 1/a_ii, restriction 0.5 V_0 + 2 V_1, prolongation +
        last sweep 1.5 V_0 + V_1 + whole FP32 rows (16 a node) + 1/a_ii;
      coarse level l: residual 3 V_l + rows, restriction V_l + 2 V_l+1,
        prolongation 2 V_l + V_l+1, sweep 3 V_l + rows (27-point rows: 32
        doubles a node on tiled levels, 27 elsewhere); coarsest: its dense
        inverse (N_c^2 doubles) and 2 V_c.
    Mixed precision (p32): the direction in FP32 takes V_0 off each iteration
    (the old p and the new p in the direction kernel). With 16 right-hand sides
    and a tiled level 1 its vectors are FP32: V_1 counts half.
    Per solve: start 3 V_0, the first V-cycle's finest residual 1.5 V_0 + rows,
    one V-cycle more than iterations, x formed from the kept directions (each
    read once, V_0 or in FP32 V_0 / 2, and x read and written), the final true
    residual 3 V_0 + rows.
    Jacobian kernels per block: J s -- dK(s) rows (80 B a node: its two
    coefficients read, 8 row entries written; the element form also reads 17 B
    a tetrahedron of connectivity and geometry class), the stencil product
    2 V_0 + rows, the output 3 V_0; J^T t -- right-hand side 2 V_0, then in the
    voxel form (Kuhn lattice of equal voxels, N_v = E / 6) the voxel sums
    2 V_0 + 128 B a voxel and the gather 128 B a voxel + 2 V_0, in the element
    form element sums 2 V_0 + 57 B a tetrahedron and gather 2 V_0 + 56 B a
    tetrahedron; output 48 B a node.
    Returns (total bytes, dict of the parts)."""
    vb = 8 * B
    V = [n * vb for n in levels]
    if B == 16 and len(levels) > 2 and levels[1] >= tiled27_min:
        V[1] //= 2   # level 1's vectors in FP32
    rows0, whole0, d0 = 64 * N, 64 * N, 8 * N
    L = len(levels)

    def coarse_rows(l):
        return (256 if levels[l] >= tiled27_min else 216) * levels[l]

    vc = 0.5 * V[0] + 2 * V[1] + 8 * levels[1]
    for l in range(1, L - 1):
        vc += 3 * V[l] + coarse_rows(l) + V[l] + 2 * V[l + 1] + 8 * levels[l + 1]      # down
        vc += 2 * V[l] + V[l + 1] + 3 * V[l] + coarse_rows(l) + 8 * levels[l]         # up
    vc += 8 * levels[-1] ** 2 + 2 * V[-1]
    vc += 1.5 * V[0] + V[1] + whole0 + d0                                             # prolongation + last sweep
    pcg_it = 3.5 * V[0] + rows0 + 3.5 * V[0] + rows0 + d0 - (1.0 * V[0] if p32 else 0.0)

    def solve(it):
        form_x = it * (0.5 if p32 else 1.0) * V[0] + 2 * V[0]
        return 3 * V[0] + 1.5 * V[0] + rows0 + d0 + (it + 1) * vc + it * pcg_it + form_x + 3 * V[0] + rows0

    if voxel:
        nv = E // 6
        jv = blocks * (80 * N + 2 * V[0] + rows0 + 3 * V[0])
        jt = blocks * (2 * V[0] + 2 * V[0] + 128 * nv) + 128 * nv + 2 * V[0] + 48 * N
    else:
        jv = blocks * (80 * N + 17 * E + 2 * V[0] + rows0 + 3 * V[0])
        jt = blocks * (2 * V[0] + 2 * V[0] + 57 * E + 2 * V[0] + 56 * E) + 48 * N
    parts = {"vcycle_per_iter": vc, "pcg_per_iter": pcg_it, "tangent_solves": blocks * solve(iters_tan),
             "adjoint_solves": blocks * solve(iters_adj), "jacobian_kernels": jv + jt}
    return parts["tangent_solves"] + parts["adjoint_solves"] + parts["jacobian_kernels"], parts


# M_delta's multigrid kernels (one right-hand side per system, two systems; profile
# counters 8-11) and their algorithmic bytes per node: the PCG's vectors of 2 N
# doubles (16 B a node), the V-cycle's finest-level vectors x0, its residual and
# z in FP32 (8 B a node), the Kuhn rows' diagonal and 7 upper entries,
# entry-major (8 entries, each read once from HBM: FP64 for the PCG product,
# FP32 for the V-cycle's finest sweeps), 1/a_ii (FP64) and the region map
# (int32). The update also writes the V-cycle's first sweep and reads 1/a_ii
# and the map.
PRIOR_MG_BYTES_PER_NODE = {
    "prior_mg_dir_spmv": ("k_mgp_dir<1,true> + k_mgp_spmv<3,1>", 8 + 4 * 16 + 2 * 8 * 8 + 2 * 4),
    "prior_mg_update": ("k_mgp_update_first<float>", 6 * 16 + 8 + 16 + 2 * 4),
    "prior_mg_resid0": ("k_mg_resid<5,1,float>", 16 + 2 * 8 + 2 * 8 * 4),
    "prior_mg_smooth0": ("k_mg_smooth<5,1,true,float>", 16 + 2 * 8 + 2 * 8 * 4 + 2 * 8),
}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (profiles/hbm_traffic.json, copy-calibrated), or None when
    the kernel source has changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    d = rec["per_dispatch_bytes"].get(kernel)
    return None if d is None else d["fetch"] + d["write"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--n-ill", type=int, default=16)
    ap.add_argument("--lsqr-steps", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=150)
    ap.add_argument("--workload", choices=("pair", "learned", "batch", "illum", "recon"), default="pair",
                    help="pair: J s + J^T t pairs at 128^3 (default); learned: the learned-guess experiment; "
                         "batch: 32 uneven instances run concurrently; illum: Algorithm 1 on an 11 mm cube "
                         "with 1, 2, 3 illuminations and data from a 2x finer mesh; recon: the whole 3 x 30 "
                         "Algorithm 1 reconstruction at 128^3")
    ap.add_argument("--instances", type=int, default=32)
    ap.add_argument("--train-phantoms", type=int, default=250,
                    help="learned workload: training phantoms (x 8 illuminations = 2000 samples)")
    ap.add_argument("--held-phantoms", type=int, default=25,
                    help="learned workload: held-out phantoms (x 8 illuminations = 200 samples)")
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--rhs-block", type=int, default=16,
                    help="recon workload: right-hand sides per block solve (1 = plain, one at a time)")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="hardware queues per process (GPU_MAX_HW_QUEUES, 1-32); 0 keeps HIP's default "
                         "(4); the batch workload's streams share these")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed",
                    help="K solves of the timed pairs: FP64 multigrid PCG, or mixed (the PCG direction in "
                         "FP32 on the tiled kernels; x, r, A p and the dots FP64)")
    ap.add_argument("--config", choices=("C1", "C2", "C3"), default="C3",
                    help="recon workload: the 16^3 face-source (C1), 64^3 (C2) or 128^3 (C3) configuration")
    ap.add_argument("--oracle-recon", action="store_true",
                    help="recon workload: also time the FP64 oracle's Algorithm 1 on the same data (C1 size)")
    ap.add_argument("--no-init", action="store_true",
                    help="skip the background fit, step 0 and TV-prior measurements")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding by illumination is described in DESIGN.md, not built)"}))
        sys.exit(2)
    if args.hw_queues:   # read by the HIP runtime when it initialises (before the first device call)
        if not 1 <= args.hw_queues <= 32:
            sys.exit("--hw-queues must be in 1..32")
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)

    import torch
    from paper_1512_02796_amd import qpat
    from qpat_inputs import make_problem, noise_draws, probe_vectors

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "illum":
        return bench_illum(args)
    if args.workload == "recon":
        return bench_recon(args)

    def d(a, dt=torch.float64):
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dt)

    t_setup = time.time()
    P = make_problem("C3", n=args.grid, n_ill=args.n_ill)
    m = P.mesh
    N, K = m.N, P.n_ill
    log(f"problem {args.grid}^3: N={N} E={m.E} n_ill={K} ({time.time() - t_setup:.1f}s)")
    prec = 1 if args.precision == "mixed" else 0
    opts = qpat.default_opts(max_rhs_block=16, precision=prec)   # multigrid-preconditioned block PCG
    ctx = qpat.Context(d(m.coords), d(m.tets, torch.int32), d(m.bfaces, torch.int32), opts=opts)
    ctx.set_sources(d(P.phi_src))
    h = torch.empty(K * N, dtype=torch.float64, device=dev)
    finfo = ctx.forward(d(P.kappa), d(P.mu), None, h)
    log("forward", finfo)
    # seeded data of the reconstruction (synthetic): chi = h + sigma |h| xi, W = 1/(sigma |h|)
    hh = h.cpu().numpy().reshape(K, N)
    sig = P.cfg["noise"]
    chi = hh + sig * np.abs(hh) * noise_draws(P.cfg["id"], K, N)
    W = 1.0 / (sig * np.abs(hh))
    s_np, t_np = probe_vectors(P.cfg["id"], K, N)
    s, t = d(s_np), d(t_np)
    Js = torch.empty(K * N, dtype=torch.float64, device=dev)
    Jt = torch.empty(2 * N, dtype=torch.float64, device=dev)

    # ---- timed J s + J^T t pairs
    for _ in range(args.warmup):
        ctx.jvp(s, Js)
        ctx.vjp(t, Jt)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append((ctx.jvp(s, Js), ctx.vjp(t, Jt)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pair_s = (t1 - t0) / args.steps
    log(f"pair: {pair_s * 1e3:.1f} ms", infos[-1])

    # ---- one more pair with per-launch HIP-event timing (no graph replay)
    ctx.profile(True)
    ctx.jvp(s, Js)
    ctx.vjp(t, Jt)
    torch.cuda.synchronize()
    ctx.profile(False)
    kst = ctx.profile_read()

    # ---- one PLSQR iteration (pair + M_delta^{-1} + reorthogonalisation)
    kt = np.log(P.kappa / P.kappa0)
    mt = np.log(P.mu / P.mu0)
    lsqr_s = prior_s = None
    ls_hist, pinfo = [], {"iters_max": None}
    if args.lsqr_steps > 0:
        ctx.prior_setup(d(kt), d(mt))
        x = torch.zeros(2 * N, dtype=torch.float64, device=dev)
        ctx.lsqr_init(d(chi), d(W), d(np.concatenate([kt, mt])), x)
        ctx.lsqr_step()                      # warm-up step
        torch.cuda.synchronize()
        ls_t0 = time.perf_counter()
        for _ in range(args.lsqr_steps):
            r, _ = ctx.lsqr_step()
            ls_hist.append(r)
        torch.cuda.synchronize()
        lsqr_s = (time.perf_counter() - ls_t0) / args.lsqr_steps
        log(f"LSQR iteration: {lsqr_s * 1e3:.1f} ms, residuals {ls_hist}")
        # M_delta^{-1} of one right-hand side: one untimed call (it captures the
        # graphs of the chunk lengths this right-hand side takes), then the mean of three
        ps, py = d(s_np), torch.empty(2 * N, dtype=torch.float64, device=dev)
        ctx.prior_solve(ps, py)
        torch.cuda.synchronize()
        p_t0 = time.perf_counter()
        for _ in range(3):
            pinfo = ctx.prior_solve(ps, py)
        torch.cuda.synchronize()
        prior_s = (time.perf_counter() - p_t0) / 3
        log(f"M_delta^-1: {prior_s * 1e3:.1f} ms", pinfo)

    # ---- the same pair one right-hand side at a time, and with the Jacobi preconditioner
    plain = None
    if not args.no_plain:
        out = {}
        for label, o in (("multigrid_fp64_one_rhs", dict(max_rhs_block=1)),
                         ("jacobi_fp64_16rhs", dict(pcg_precond=0, precision=0)),
                         ("jacobi_mixed_16rhs", dict(pcg_precond=0, precision=1))):
            ctx.set_opts(**o)
            ctx.forward(d(P.kappa), d(P.mu), None, None)     # hierarchy / operator for these options
            torch.cuda.synchronize()
            a = time.perf_counter()
            i1 = ctx.jvp(s, Js)
            i2 = ctx.vjp(t, Jt)
            torch.cuda.synchronize()
            dt = time.perf_counter() - a
            out[label] = {"pairs_per_s": round(1.0 / dt, 4), "ms_per_pair": round(dt * 1e3, 2),
                          "pcg_iters_sum": i1["iters_sum"] + i2["iters_sum"],
                          "pcg_iters_max": max(i1["iters_max"], i2["iters_max"])}
            log(label, out[label])
        ctx.set_opts(max_rhs_block=16, pcg_precond=1, precision=prec)
        plain = out

    # ---- mixed precision (FP32 operator and vectors in Jacobi-PCG K solves, FP64
    # dots, reliable updates and LSQR) against the FP64 multigrid path: seconds per
    # PLSQR iteration from the same start, and the final LSQR residuals
    precision_cmp = None
    if args.lsqr_steps > 0 and not args.no_plain:
        precision_cmp = {}
        beta_lin = d(np.concatenate([kt, mt]))
        for label, o in (("fp64_multigrid", dict(pcg_precond=1, precision=0)),
                         ("mixed_multigrid", dict(pcg_precond=1, precision=1)),
                         ("mixed_jacobi", dict(pcg_precond=0, precision=1))):
            ctx.set_opts(max_rhs_block=16, **o)
            ctx.forward(d(P.kappa), d(P.mu), None, None)
            ctx.prior_setup(d(kt), d(mt))
            x = torch.zeros(2 * N, dtype=torch.float64, device=dev)
            ctx.lsqr_init(d(chi), d(W), beta_lin, x)
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(args.lsqr_steps):
                r, _ = ctx.lsqr_step()
            torch.cuda.synchronize()
            precision_cmp[label] = {"s_per_lsqr_iter": round((time.perf_counter() - a) / args.lsqr_steps, 4),
                                    "final_lsqr_residual": r, "steps": args.lsqr_steps}
        ctx.set_opts(max_rhs_block=16, pcg_precond=1, precision=prec)
        ctx.forward(d(P.kappa), d(P.mu), None, None)
        r64 = precision_cmp["fp64_multigrid"]["final_lsqr_residual"]
        for label in ("mixed_multigrid", "mixed_jacobi"):
            rr = precision_cmp[label]["final_lsqr_residual"]
            precision_cmp[label]["final_residual_rel_diff_vs_fp64"] = abs(rr - r64) / r64
        log("precision", precision_cmp)

    # ---- calibration copy for HBM counters (profiling runs only)
    if args.copy_calib_mib:
        a = torch.empty(args.copy_calib_mib * (1 << 20) // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    # ---- Algorithm 1's initialisation (background fit, step 0) and the TV prior
    init = None
    if not args.no_init and args.lsqr_steps > 0:
        init = {}
        torch.cuda.synchronize()
        a = time.perf_counter()
        k0, m0, fit_it, finf = ctx.fit_background(d(chi), d(W), 1.5 * P.kappa0, 0.7 * P.mu0)
        torch.cuda.synchronize()
        init["fit_s"] = round(time.perf_counter() - a, 4)
        init["fit"] = {"start": [1.5 * P.kappa0, 0.7 * P.mu0], "kappa0": k0, "mu0": m0, "gauss_newton_iters": fit_it,
                       "pcg_solves": finf["n_solves"], "pcg_iters_sum": finf["iters_sum"]}
        beta0 = torch.zeros(2 * N, dtype=torch.float64, device=dev)
        ctx.init_guess(d(chi), m0, beta0)                  # the context is at the fitted pair
        ctx.forward_log(k0, m0, beta0)
        ctx.prior_setup(beta0[:N], beta0[N:])
        x0 = torch.zeros(2 * N, dtype=torch.float64, device=dev)
        ctx.lsqr_init_kappa(d(chi), d(W), beta0, x0)
        ctx.lsqr_step()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.lsqr_steps):
            ctx.lsqr_step()
        torch.cuda.synchronize()
        init["step0_s_per_iter"] = round((time.perf_counter() - a) / args.lsqr_steps, 4)
        ctx.prior_setup_r(d(kt), d(mt), qpat.PRIOR_TVQ, 5e-3, 1.0)
        torch.cuda.synchronize()
        a = time.perf_counter()
        tinf = ctx.prior_solve(d(s_np), torch.empty(2 * N, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        init["tv_prior_solve_s"] = round(time.perf_counter() - a, 4)
        init["tv_prior_iters"] = tinf["iters_max"]
        log("initialisation", init)

    # ---- measured bandwidth ceiling: STREAM triad a = b + s c in FP64 (3 x 512 MiB)
    n_tr = (512 << 20) // 8
    tb = torch.ones(n_tr, dtype=torch.float64, device=dev)
    tc = torch.ones_like(tb)
    ta = torch.empty_like(tb)
    for _ in range(2):
        torch.add(tb, tc, alpha=3.0, out=ta)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.add(tb, tc, alpha=3.0, out=ta)
    e1.record()
    torch.cuda.synchronize()
    triad_gbs = 3 * n_tr * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ta, tb, tc

    # ---- roofline of the dominant kernel (live HIP-event timing)
    layout = ctx.operator_layout()
    timed = {k: kst[k] for k in MG_KERNELS if kst[k]["launches"]}
    key = max(timed, key=lambda k: timed[k]["total_ms"])
    st = timed[key]
    p32 = prec == 1
    name = mg_kernel(key, kst, p32)[0]
    bytes_total = mg_algorithmic_bytes(key, N, layout, st, kst, p32)
    avg_ms = st["total_ms"] / st["launches"]
    achieved = bytes_total / st["launches"] / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_ms": round(avg_ms, 4), "launches": st["launches"],
                "bytes_per_launch": round(bytes_total / st["launches"]),
                "operator": "stencil (diagonal + %d upper offsets)" % (layout["stencil_arrays"] - 1),
                "other_kernels": {mg_kernel(k, kst, p32)[0]: {
                    "avg_ms": round(v["total_ms"] / v["launches"], 4), "launches": v["launches"],
                    "GB/s": round(mg_algorithmic_bytes(k, N, layout, v, kst, p32) / v["total_ms"] / 1e6, 1)}
                    for k, v in timed.items() if k != key}}
    roofline["traffic"] = measured_traffic(name)
    roofline["stream_triad_GBs"] = round(triad_gbs, 1)
    roofline["frac_of_triad"] = round(achieved / triad_gbs, 4)
    log("roofline", roofline)

    # ---- the whole pair against the HBM roofline: algorithmic bytes of every kernel
    n1 = args.grid + 1
    levels = mg_levels(n1, n1, n1)
    it_t, it_a = infos[-1][0]["iters_max"], infos[-1][1]["iters_max"]
    blocks = (K + 15) // 16
    pb, parts = pair_algorithmic_bytes(N, m.E, levels, 16, blocks, it_t, it_a, p32=prec == 1)
    roofline["pair"] = {"bytes": round(pb), "GB_per_s": round(pb / pair_s / 1e9, 1),
                        "frac": round(pb / pair_s / 1e9 / HBM_PEAK_GBS, 4),
                        "frac_of_triad": round(pb / pair_s / 1e9 / triad_gbs, 4),
                        "levels": levels, "pcg_iters": [it_t, it_a],
                        "bytes_per_iteration": round(parts["vcycle_per_iter"] + parts["pcg_per_iter"]),
                        "jacobian_kernels_bytes": round(parts["jacobian_kernels"])}
    log("pair roofline", roofline["pair"])
    try:   # z-chunk lengths of the tiled kernels (autotuned or the cost model's)
        roofline["tile_schedule"] = ctx.tile_schedule(16)
        log("tile schedule", roofline["tile_schedule"])
    except Exception as e:   # no 16-right-hand-side tiling on this mesh
        log("tile schedule", str(e))

    # ---- M_delta^{-1}'s multigrid kernels (one right-hand side per system)
    if args.lsqr_steps > 0:
        ctx.profile(True)
        ctx.prior_solve(d(s_np), torch.empty(2 * N, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        ctx.profile(False)
        pst = ctx.profile_read()
        pk = {}
        for key, (kname, bpn) in PRIOR_MG_BYTES_PER_NODE.items():
            v = pst[key]
            if v["launches"]:
                avg = v["total_ms"] / v["launches"]
                gbs = bpn * N / (avg * 1e-3) / 1e9
                pk[kname] = {"avg_ms": round(avg, 4), "launches": v["launches"], "bytes_per_launch": bpn * N,
                             "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
        roofline["prior_kernels"] = pk
        log("M_delta kernels", pk)

    # ---- CPU oracle on a bounded sample of the same system, and a whole oracle
    # pair at the 16^3 workload beside the GPU's
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(P, args.cpu_iters, plain)
        cpu["measured_pair_16cube"] = small_pair_both_sides(ctx_factory=lambda Q: qpat.Context(
            d(Q.mesh.coords), d(Q.mesh.tets, torch.int32), d(Q.mesh.bfaces, torch.int32),
            opts=qpat.default_opts(max_rhs_block=16)), d=d)
        log("cpu_baseline", cpu)

    ctx.close()
    res = {
        "metric": METRIC,
        "value": round(1.0 / pair_s, 4),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(pair_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f64 (PCG direction stored f32)",
        "data": "synthetic",
        "config": {"workload": f"QPAT J s + J^T t pair, {args.grid}^3 Kuhn voxels (N={N}, E={m.E}), "
                               f"{K} Gaussian illuminations, seeded ellipsoid phantom, 16-RHS block PCG "
                               "with a geometric-multigrid V-cycle, "
                               + ("FP64" if prec == 0 else "mixed (direction FP32; x, r, A p, dots FP64)")
                               + ", true residual <= 1e-10 ||b|| in FP64",
                   "grid": args.grid, "nodes": N, "tets": m.E, "n_ill": K, "precision": args.precision,
                   "preconditioner": "multigrid V(1,1), weighted Jacobi, Galerkin coarse levels",
                   "rhs_block": 16, "pcg_rtol": 1e-10},
        "s_per_lsqr_iter": round(lsqr_s, 4) if lsqr_s else None,
        "prior_solve_s": round(prior_s, 4) if prior_s else None,
        "pcg_iters": {"pair_sum": infos[-1][0]["iters_sum"] + infos[-1][1]["iters_sum"],
                      "tangent_max": infos[-1][0]["iters_max"], "adjoint_max": infos[-1][1]["iters_max"],
                      "prior": pinfo["iters_max"]},
        "plain": plain,
        "precision": precision_cmp,
        "init": init,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def bench_learned(args):
    """Learned PCG initial guess on the 96^3 workload with 8 Gaussian
    illuminations: train on solver-generated samples (phantoms x
    illuminations), then on held-out phantoms compare the forward block
    solve from zero, from the homogeneous fluence, and from the network's
    prediction (same true-residual tolerance 1e-10)."""
    import torch
    from paper_1512_02796_amd import qpat, learned
    from qpat_inputs import make_problem, initial_params
    dev = torch.device("cuda:0")
    P = make_problem("C5")
    m = P.mesh
    N, K = m.N, P.n_ill
    ctx = qpat.Context(torch.as_tensor(m.coords, device=dev), torch.as_tensor(m.tets, device=dev),
                       torch.as_tensor(m.bfaces, device=dev),
                       opts=qpat.default_opts(max_rhs_block=8))
    ctx.set_sources(torch.as_tensor(P.phi_src, device=dev))
    n1 = m.n + 1
    ctx.guess_setup(n1, n1, n1)
    ctx.guess_set_params(torch.as_tensor(initial_params(P.cfg["id"]), device=dev))
    phi_hom = learned.homogeneous_fluence(ctx, P.kappa0, P.mu0, dev)
    t0 = time.time()
    train = learned.make_samples(ctx, m, args.train_phantoms, P.cfg["id"], 3, dev)
    held = learned.make_samples(ctx, m, args.held_phantoms, P.cfg["id"], 4, dev)
    t_data = time.time() - t0
    log(f"data: {len(train) * K} training and {len(held) * K} held-out samples in {t_data:.1f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = learned.train(ctx, train, phi_hom, P.kappa0, P.mu0, args.epochs, 1e-3, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = args.epochs * len(train) * K
    agg, _ = learned.evaluate(ctx, held, phi_hom, P.kappa0, P.mu0, dev)
    log("held-out", agg)
    # conv MFMA throughput: forward 2 V (27 (3 16) + 2 (27 16 16) + 27 16) flop per sample,
    # a training step is forward + weight gradients + input gradients of layers 2-4 (~3x forward)
    fwd_flop = 2.0 * N * 27 * (3 * 16 + 16 * 16 * 2 + 16)
    train_tflops = 3.0 * fwd_flop * steps / t_train / 1e12
    ctx.close()
    res = {
        "metric": "forward PCG iterations and wall time to rtol 1e-10, learned vs zero initial guess",
        "value": round(agg["zero_ms"] / agg["net_ms"], 4),
        "unit": "x speed-up of the forward block solve (zero start / learned start)",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": round(t_train / steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16/f32 net, f64 solve",
        "data": "synthetic",
        "config": {"workload": f"learned PCG initial guess, {m.n}^3 Kuhn voxels (N={N}), {K} Gaussian "
                               f"illuminations, 4-layer 3x3x3 conv net 3-16-16-16-1, "
                               f"{len(train) * K} training / {len(held) * K} held-out samples, "
                               f"{args.epochs} epochs Adam"},
        "pcg_iters_per_solve": {"zero": agg["zero_iters"], "homogeneous_fluence": agg["hom_iters"],
                                "learned": agg["net_iters"]},
        "ms_per_block_solve": {"zero": agg["zero_ms"], "homogeneous_fluence": agg["hom_ms"],
                               "learned_incl_inference": agg["net_ms"]},
        "train": {"seconds": round(t_train, 2), "loss_per_epoch": hist, "data_seconds": round(t_data, 1),
                  "approx_TFLOP_s": round(train_tflops, 1), "peak_bf16_TFLOP_s": 2500.0},
        "max_relres": agg["relres"],
    }
    print(json.dumps(res), flush=True)


def bench_recon(args):
    """The whole Algorithm 1 run of the 128^3 workload: 16 Gaussian illuminations,
    seeded ellipsoid phantom, 2% noise, 3 outer steps of 30 PLSQR steps each from the
    configured background (fixed counts, as configured), FP64 multigrid block PCG.
    Reports the mean time per PLSQR iteration over all 90 (forward solves, prior
    set-ups and the step-4 checks included in the total) and the residual history."""
    import torch
    from paper_1512_02796_amd import qpat
    from paper_1512_02796_amd.driver import reconstruct
    from qpat_inputs import make_problem, noise_draws
    dev = torch.device("cuda:0")

    def d(a, dt=torch.float64):
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dt)

    P = make_problem("C3", n=args.grid, n_ill=args.n_ill) if args.config == "C3" else make_problem(args.config)
    m = P.mesh
    N, K = m.N, P.n_ill
    ctx = qpat.Context(d(m.coords), d(m.tets, torch.int32), d(m.bfaces, torch.int32),
                       opts=qpat.default_opts(max_rhs_block=16))
    ctx.set_sources(d(P.phi_src))
    h = torch.empty(K * N, dtype=torch.float64, device=dev)
    ctx.forward(d(P.kappa), d(P.mu), None, h)
    src = "face" if P.cfg["source"] == "face" else "Gaussian"
    hh = h.cpu().numpy().reshape(K, N)
    sig = P.cfg["noise"]
    chi = hh + sig * np.abs(hh) * noise_draws(P.cfg["id"], K, N)
    W = 1.0 / (sig * np.abs(hh))
    outer, inner = P.cfg["outer"], P.cfg["inner"]
    ctx.set_opts(max_rhs_block=args.rhs_block)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    beta, lg = reconstruct(ctx, d(chi), d(W), P.kappa0, P.mu0, outer=outer, inner=inner)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    steps = sum(len(hst) - 1 for hst in lg["lsqr"])
    b = beta.cpu().numpy()
    kap = P.kappa0 * np.exp(b[:N])
    mu = P.mu0 * np.exp(b[N:])
    out = {"seconds": round(total, 3), "lsqr_steps": steps, "s_per_lsqr_iter": round(total / steps, 4),
           "res_nl": [round(r, 1) for r in lg["res_nl"]], "sqrt_n_data": round(float(np.sqrt(K * N)), 1),
           "final_lsqr_residuals": [round(hst[-1], 2) for hst in lg["lsqr"]],
           "pcg_iters_per_outer": lg["pcg_iters"], "rejected": lg["rejected"],
           "rel_err_kappa": round(float(np.linalg.norm(kap - P.kappa) / np.linalg.norm(P.kappa)), 4),
           "rel_err_mu": round(float(np.linalg.norm(mu - P.mu) / np.linalg.norm(P.mu)), 4)}
    log("reconstruction", out)
    ctx.close()
    if args.oracle_recon:
        # the FP64 oracle's Algorithm 1 on the same data (sparse LU for K and M_delta)
        from oracle import fem
        from oracle.driver import reconstruct as oracle_reconstruct
        g = fem.geometry(m.coords, m.tets, m.bfaces)
        a = time.perf_counter()
        ob, olg = oracle_reconstruct(g, P.phi_src, chi, W, P.kappa0, P.mu0, outer, inner)
        osec = time.perf_counter() - a
        osteps = sum(len(hst) - 1 for hst in olg["lsqr"])
        out["oracle"] = {"seconds": round(osec, 3), "s_per_lsqr_iter": round(osec / osteps, 4), "cores": 1,
                         "final_lsqr_residuals": [round(hst[-1], 2) for hst in olg["lsqr"]],
                         "res_nl": [round(r, 1) for r in olg["res_nl"]],
                         "gpu_speedup": round(osec / total, 1)}
        log("oracle reconstruction", out["oracle"])
    n_vox = m.n
    res = {"metric": f"seconds per PLSQR iteration over the whole Algorithm 1 reconstruction at {n_vox}^3",
           "value": out["s_per_lsqr_iter"], "unit": "s", "n_gpus": 1, "steps": steps, "warmup": 0,
           "ms_per_step": round(total / steps * 1e3, 2), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"Algorithm 1, {n_vox}^3 Kuhn voxels (N={N}), {K} {src} illuminations, "
                                  f"seeded phantom, {round(100 * sig)}% noise, {outer} x {inner} PLSQR steps, FP64 "
                                  f"multigrid PCG, {args.rhs_block} right-hand side(s) per block solve",
                      "rhs_block": args.rhs_block, "config": args.config},
           "reconstruction": out}
    print(json.dumps(res), flush=True)


def bench_illum(args):
    """Illumination study (Sec. 5, second test; its inclusion sizes are not given,
    so seeded ellipsoids): an 11 mm cube at 32^3 voxels, two inclusions, 1% noise on
    data simulated on the 64^3 mesh and read at the 32^3 nodes (no inverse crime).
    Algorithm 1 with the background fit, the initial guess, step 0 and 3 outer steps
    of at most 30 PLSQR steps (window rule m0 = 10, tau = 1e-2), for 1, 2 and 3
    face illuminations (-z; -z, +z; -z, +z, -x); relative errors of kappa and mu."""
    import torch
    from paper_1512_02796_amd import qpat
    from paper_1512_02796_amd.driver import finer_mesh_data, reconstruct
    from qpat_inputs import make_problem, noise_draws, coarse_in_fine
    dev = torch.device("cuda:0")

    def d(a, dt=torch.float64):
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dt)

    def context(m, P):
        c = qpat.Context(d(m.coords), d(m.tets, torch.int32), d(m.bfaces, torch.int32), opts=qpat.default_opts())
        c.set_sources(d(P.phi_src))
        return c

    out, times = {}, []
    n = 32
    for k in (1, 2, 3):
        P, Pf = make_problem("S2", n=n, n_ill=k), make_problem("S2", n=2 * n, n_ill=k)
        cf = context(Pf.mesh, Pf)
        h = finer_mesh_data(cf, d(Pf.kappa), d(Pf.mu), d(coarse_in_fine(n), torch.int64))
        cf.close()
        N = P.mesh.N
        sig = P.cfg["noise"]
        hh = h.cpu().numpy()
        chi = hh + sig * np.abs(hh) * noise_draws(P.cfg["id"], k, N)
        W = 1.0 / (sig * np.abs(hh))
        ctx = context(P.mesh, P)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        beta, lg = reconstruct(ctx, d(chi), d(W), P.kappa0, P.mu0, outer=3, inner=30, m0=10, tau=1e-2,
                               fit=True, step0_inner=30)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        b = beta.cpu().numpy()
        kap = lg["kappa0"] * np.exp(b[:N])
        mu = lg["mu0"] * np.exp(b[N:])
        out[k] = {"seconds": round(dt, 3), "kappa0": lg["kappa0"], "mu0": lg["mu0"],
                  "rel_err_kappa": round(float(np.linalg.norm(kap - P.kappa) / np.linalg.norm(P.kappa)), 4),
                  "rel_err_mu": round(float(np.linalg.norm(mu - P.mu) / np.linalg.norm(P.mu)), 4),
                  "rel_err_mu_background": round(float(np.linalg.norm(lg["mu0"] - P.mu) / np.linalg.norm(P.mu)), 4),
                  "lsqr_steps": [len(x) - 1 for x in lg["lsqr"]], "step0_steps": len(lg["step0"]) - 1,
                  "res_nl": [round(r, 2) for r in lg["res_nl"]], "sqrt_n_data": round(float(np.sqrt(k * N)), 1)}
        log(f"{k} illumination(s)", out[k])
        ctx.close()
    res = {"metric": "seconds per Algorithm 1 reconstruction (fit, step 0, 3 outer steps), 11 mm cube",
           "value": round(float(np.mean(times)), 3), "unit": "s", "n_gpus": 1, "steps": 3, "warmup": 0,
           "ms_per_step": round(float(np.mean(times)) * 1e3, 1), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"11 mm cube, {n}^3 Kuhn voxels (N={(n + 1) ** 3}), data on {2 * n}^3, "
                                  "two seeded ellipsoids, 1% noise, 1/2/3 face illuminations"},
           "by_illuminations": out}
    print(json.dumps(res), flush=True)


def bench_batch(args):
    """Uneven batched instances: `--instances` independent reconstructions
    (n ~ U{24..96} voxels per side, 4..12 Gaussian illuminations, seeded
    ellipsoid phantoms), each a context on its own HIP stream, advanced
    together by qpat_batch (one host thread per instance). Reports aggregate
    J s + J^T t pairs/s, seconds per batched PLSQR step (every instance one
    step), and the same pairs run one instance after another."""
    import torch
    from paper_1512_02796_amd import qpat
    from qpat_inputs import make_problem, batch_instances, probe_vectors
    dev = torch.device("cuda:0")

    def d(a):
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float64)

    t0 = time.time()
    inst = batch_instances(args.instances)
    ctxs, streams, P_all, S, T, JS, JT, kap, mus = [], [], [], [], [], [], [], [], []
    for spec in inst:
        P = make_problem("C4", n=spec["n"], n_ill=spec["n_ill"], id=spec["id"])
        m = P.mesh
        st = torch.cuda.Stream(device=dev)
        opts = qpat.default_opts(precision=1 if args.precision == "mixed" else 0, max_rhs_block=16,
                                 lsqr_max_steps=8)
        ctx = qpat.Context(d(m.coords), d(m.tets).to(torch.int32), d(m.bfaces).to(torch.int32), opts=opts,
                           stream=st)
        ctx.set_sources(d(P.phi_src))
        s_np, t_np = probe_vectors(spec["id"], P.n_ill, m.N)
        ctxs.append(ctx)
        streams.append(st)
        P_all.append(P)
        S.append(d(s_np))
        T.append(d(t_np))
        JS.append(torch.empty(P.n_ill * m.N, dtype=torch.float64, device=dev))
        JT.append(torch.empty(2 * m.N, dtype=torch.float64, device=dev))
        kap.append(d(P.kappa))
        mus.append(d(P.mu))
    torch.cuda.synchronize()
    nodes = sum(P.mesh.N for P in P_all)
    log(f"{len(ctxs)} instances, {nodes} nodes, {sum(P.n_ill for P in P_all)} illuminations "
        f"({time.time() - t0:.1f}s setup)")
    H = [torch.empty(P.n_ill * P.mesh.N, dtype=torch.float64, device=dev) for P in P_all]
    qpat.batch(ctxs, "forward", in0=kap, in1=mus, out0=H)
    qpat.batch(ctxs, "pair", in0=S, out0=JS, in1=T, out1=JT)          # warm-up (graphs, occupancy)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(args.steps):
        infos = qpat.batch(ctxs, "pair", in0=S, out0=JS, in1=T, out1=JT)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - a) / args.steps
    log(f"batched round of {len(ctxs)} pairs: {t_batch * 1e3:.1f} ms")
    # the same pairs one instance after another
    a = time.perf_counter()
    for _ in range(args.steps):
        for i, ctx in enumerate(ctxs):
            ctx.jvp(S[i], JS[i])
            ctx.vjp(T[i], JT[i])
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - a) / args.steps
    log(f"sequential round: {t_seq * 1e3:.1f} ms")
    # PLSQR: each instance initialised at its true phantom, then batched steps
    lsqr_s = None
    if args.lsqr_steps > 0:
        for i, (ctx, P) in enumerate(zip(ctxs, P_all)):
            kt = np.log(P.kappa / P.kappa0)
            mt = np.log(P.mu / P.mu0)
            ctx.prior_setup(d(kt), d(mt))
            hh = H[i].cpu().numpy().reshape(P.n_ill, P.mesh.N)
            chi = hh * (1.0 + P.cfg["noise"] * np.random.default_rng(P.cfg["id"]).standard_normal(hh.shape))
            W = 1.0 / (P.cfg["noise"] * np.abs(hh))
            ctx.lsqr_init(d(chi), d(W), d(np.concatenate([kt, mt])),
                          torch.zeros(2 * P.mesh.N, dtype=torch.float64, device=dev))
        qpat.batch(ctxs, "lsqr_step")
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.lsqr_steps):
            qpat.batch(ctxs, "lsqr_step")
        torch.cuda.synchronize()
        lsqr_s = (time.perf_counter() - a) / args.lsqr_steps
        log(f"batched PLSQR step: {lsqr_s * 1e3:.1f} ms")
    for c in ctxs:
        c.close()
    res = {
        "metric": "aggregate J s + J^T t pairs/s over uneven batched instances",
        "value": round(len(ctxs) / t_batch, 4),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (PCG direction stored f32)",
        "data": "synthetic",
        "config": {"workload": f"{len(ctxs)} instances, n ~ U{{24..96}}^3 Kuhn voxels ({nodes} nodes in all), "
                               f"4-12 Gaussian illuminations each, {args.precision} multigrid 16-RHS block PCG, "
                               f"rtol 1e-10, one stream and host thread per instance",
                   "instances": len(ctxs), "nodes_total": nodes, "precision": args.precision,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "sequential_ms_per_round": round(t_seq * 1e3, 3),
        "batched_speedup": round(t_seq / t_batch, 3),
        "s_per_batched_lsqr_step": round(lsqr_s, 4) if lsqr_s else None,
        "pcg_iters_sum": int(sum(i["iters_sum"] for i in infos)),
    }
    print(json.dumps(res), flush=True)


def small_pair_both_sides(ctx_factory, d, reps=20):
    """One J s + J^T t pair at the 16^3 face-source workload (N = 4913, 4
    illuminations), timed whole on the FP64 oracle (sparse LU factorisation of
    K untimed, as the GPU's forward solve is; the first products form the
    Appendix's G(1), G(2) matrices, which is how the oracle applies J) and on
    the GPU (median of `reps` pairs after a warm-up)."""
    import torch
    from qpat_inputs import make_problem, probe_vectors
    from oracle import fem
    from oracle.jacobian import Linearisation
    Q = make_problem("C1")
    g = fem.geometry(Q.mesh.coords, Q.mesh.tets, Q.mesh.bfaces)
    lin = Linearisation(g, Q.kappa, Q.mu, Q.phi_src)
    s, t = probe_vectors(Q.cfg["id"], Q.n_ill, g.N)
    a = time.perf_counter()
    lin.jvp(s)
    lin.vjp(t)
    oracle_s = time.perf_counter() - a
    ctx = ctx_factory(Q)
    ctx.set_sources(d(Q.phi_src))
    ctx.forward(d(Q.kappa), d(Q.mu))
    Js = torch.empty(Q.n_ill * g.N, dtype=torch.float64, device="cuda")
    Jt = torch.empty(2 * g.N, dtype=torch.float64, device="cuda")
    sd, td = d(s), d(t)
    ctx.jvp(sd, Js)
    ctx.vjp(td, Jt)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        ctx.jvp(sd, Js)
        ctx.vjp(td, Jt)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    ctx.close()
    gpu_s = float(np.median(ts))
    return {"workload": "16^3 Kuhn voxels (N=4913), 4 face illuminations, J s + J^T t, FP64",
            "oracle_s": round(oracle_s, 4), "oracle_cores": 1, "gpu_s": round(gpu_s, 5),
            "gpu_over_oracle": round(oracle_s / gpu_s, 1)}


def cpu_baseline(P, iters, plain):
    """FP64 oracle on the same 128^3 system: Jacobi-PCG iterations of one
    right-hand side (the oracle's K solve), timed over `iters` iterations and
    scaled to one J s + J^T t pair by the pair's Jacobi-PCG iteration count
    in FP64 (the oracle's algorithm; measured on the GPU)."""
    from oracle import fem
    from oracle.solve import pcg
    m = P.mesh
    a = time.time()
    g = fem.geometry(m.coords, m.tets, m.bfaces)
    Kmat = fem.system_matrix(g, P.kappa, P.mu)
    f = fem.load_vectors(g, P.phi_src[:1])[0]
    setup = time.time() - a
    t0 = time.perf_counter()
    try:
        pcg(Kmat, f, rtol=1e-30, maxit=iters)
    except RuntimeError:
        pass                              # stopped at maxit by design
    dt = (time.perf_counter() - t0) / iters
    pair_iters = plain["jacobi_fp64_16rhs"]["pcg_iters_sum"] if plain else None
    out = {"kind": "oracle", "cores": 1, "unit": "pairs/s",
           "sample": f"oracle Jacobi-PCG on the {m.n}^3 K system, {iters} iterations of one right-hand side "
                     f"({dt * 1e3:.1f} ms/iteration, single-threaded scipy/numpy; assembly {setup:.0f}s untimed)",
           "s_per_pcg_iter": round(dt, 5)}
    if pair_iters:
        out["value"] = round(1.0 / (dt * pair_iters), 6)
        out["sample"] += (f", scaled by the {pair_iters} Jacobi-PCG iterations (the oracle's solver) of one pair "
                          "(32 solves, FP64, measured on the GPU)")
    else:
        out["value"] = None
    return out


if __name__ == "__main__":
    main()
