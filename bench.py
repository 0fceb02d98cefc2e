"""Krylov vectors per second at 200^3 on one MI355X.

One step = one Krylov vector (eqs. 8-10): the linearized momentum stencil, the
SIMPLE projection (divergence, tensor-product pressure-correction solve (TPT unless
--poisson tpf), velocity/pressure correction, divergence certificate) to a relative divergence
residual rho <= 1e-8, on a 200^3 tanh-stretched grid (centre/wall spacing 10),
Re = 1900, lid along x.  Inputs are seeded (SplitMix64) and resident in HBM
before the timed region.  Three forms: plain FP64, mixed (FP32 solves inside
FP64 refinement) and learned (a BF16 U-Net's guess of the first correction,
trained beforehand on a 64^3 grid with pairs the method generates, then mixed
passes).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--size 200] [--no-cpu]
                    [--train-steps 300] [--poisson tpt|tpf]
    python bench.py --planes | --critical N[,N...] [--alpha 0|45] | --learned-recipe PAIRS
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
# multiply-adds x 2 per voxel of the network's padded grid: 3x3x3 convs 4->16, 16->32 (1/8 of
# the voxels), 32->64 (1/64), 96->32 (1/8), 48->16, and the 16->1 head
NN_FLOP_PER_VOXEL = 2.0 * (27 * 4 * 16 + 27 * 16 * 32 / 8 + 27 * 32 * 64 / 64 + 27 * 96 * 32 / 8 + 27 * 48 * 16 + 16)
RE = 1900.0
TANH_RATIO = 10.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-reps", type=int, default=3, help="timed oracle Krylov vectors (after one warm-up)")
    ap.add_argument("--train-steps", type=int, default=300, help="Adam steps of the learned guess (64^3 pairs)")
    ap.add_argument("--train-size", type=int, default=64)
    ap.add_argument("--critical", type=str, default="", metavar="N[,N...]",
                    help="instead of the Krylov-vector benchmark: critical Reynolds number of the N^3 cube "
                         "on the sine grid of eq. 5, lid at --alpha (Newton continuation, then the secant "
                         "driver lc_critical_re); one JSON line")
    ap.add_argument("--alpha", type=float, choices=(0.0, 45.0), default=0.0,
                    help="lid angle (degrees) of --critical: 0 (parallel to a side wall) or 45 (diagonal)")
    ap.add_argument("--base-flow", choices=("steady", "seeded"), default="steady",
                    help="benchmark base flow: the Newton steady state (continued at 100^3, prolongated, "
                         "Newton at the benchmark grid) or a seeded divergence-free field (faster set-up; the "
                         "cost of a Krylov vector does not depend on U)")
    ap.add_argument("--poisson", choices=("tpt", "tpf"), default="tpt",
                    help="pressure-solve route (transforms along y, z with tridiagonal solves along x, "
                         "or transforms along x, y, z)")
    ap.add_argument("--learned-recipe", type=int, default=0, metavar="PAIRS",
                    help="instead of the Krylov-vector benchmark: train the learned guess on PAIRS pairs "
                         "from 64^3 and 100^3 Newton steady states (Re 1000-2500, both lid directions) and "
                         "evaluate it inside SIMPLE at 150^3 and 200^3; one JSON line")
    ap.add_argument("--save-net", type=str, default="", metavar="PATH",
                    help="with --learned-recipe: write the trained parameters to PATH (lc_net_save)")
    ap.add_argument("--planes", action="store_true",
                    help="instead of the Krylov-vector benchmark: only the plane projections and potentials "
                         "(eqs. 11-17) at --size^3; one JSON line")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(ctx, torch, n_vec, seed0=1):
    """v_s = P(r_s)/|P(r_s)| with r_s uniform [-1, 1) on interior faces (seeded)."""
    import synth
    vs = []
    for s in range(seed0, seed0 + n_vec):
        r = torch.from_numpy(synth.random_velocity(ctx.nx, ctx.ny, ctx.nz, s)).cuda()
        v, _, st = ctx.project(r, tol=1e-12, max_iter=4)
        v /= torch.linalg.vector_norm(v)
        vs.append(v)
    return vs


def synthetic_base_flow(ctx, torch):
    """A seeded divergence-free field with max |U| = 1 (the Krylov-vector cost
    does not depend on the values of U)."""
    import synth
    r = torch.from_numpy(synth.random_velocity(ctx.nx, ctx.ny, ctx.nz, 1000)).cuda()
    U, _, _ = ctx.project(r, tol=1e-12, max_iter=4)
    U /= U.abs().max()
    return U


def _interp_axis(a, old, new, axis):
    """Linear interpolation of array a along `axis` from positions old to new (clamped
    beyond the end positions)."""
    import numpy as np
    q = np.clip(np.searchsorted(old, new) - 1, 0, len(old) - 2)
    t = np.clip((new - old[q]) / (old[q + 1] - old[q]), 0.0, 1.0)
    shape = [1] * a.ndim
    shape[axis] = len(new)
    t = t.reshape(shape)
    return np.take(a, q, axis=axis) * (1.0 - t) + np.take(a, q + 1, axis=axis) * t


def prolongate_velocity(U, coarse, fine):
    """A staggered velocity (packed u|v|w) of the coarse grid interpolated to the fine one:
    each component separably linear between its own positions (faces along its direction,
    cell centres across)."""
    import numpy as np
    (cx, cy, cz), (fx, fy, fz) = coarse, fine
    nx, ny, nz = len(cx) - 1, len(cy) - 1, len(cz) - 1
    c = lambda f: 0.5 * (f[1:] + f[:-1])
    u = U[:(nx + 1) * ny * nz].reshape(nz, ny, nx + 1)
    v = U[(nx + 1) * ny * nz:(nx + 1) * ny * nz + nx * (ny + 1) * nz].reshape(nz, ny + 1, nx)
    w = U[(nx + 1) * ny * nz + nx * (ny + 1) * nz:].reshape(nz + 1, ny, nx)
    out = []
    for a, (px, py, pz), (qx, qy, qz) in ((u, (cx, c(cy), c(cz)), (fx, c(fy), c(fz))),
                                        (v, (c(cx), cy, c(cz)), (c(fx), fy, c(fz))),
                                        (w, (c(cx), c(cy), cz), (c(fx), c(fy), fz))):
        a = _interp_axis(a, px, qx, 2)
        a = _interp_axis(a, py, qy, 1)
        a = _interp_axis(a, pz, qz, 0)
        out.append(a.ravel())
    return np.concatenate(out)


def steady_base_flow(lk, torch, ctx, coarse=100):
    """The benchmark's base flow: the Newton steady state of the coarse^3 grid (continued from
    rest with Stokes-preconditioned Newton), prolongated to ctx's grid, projected onto the
    divergence-free space and taken to the steady state there by Newton.  Returns (U, info)."""
    t0 = time.perf_counter()
    cc = lk.Context(coarse)
    cc.set_stretching("tanh", TANH_RATIO)
    cc.set_lid(0.0)
    cc.set_base_flow(torch.zeros(cc.nvel, dtype=torch.float64, device="cuda"))
    cc.set_stokes_precond(float("inf"))
    for re in (250.0, 500.0, 800.0, 1100.0, 1400.0, 1600.0, 1750.0, 1850.0, RE):
        cc.set_re(re)
        hist = cc.newton(tol=1e-11, max_steps=12, lin_tol=1e-8, gmres_m=100, max_vectors=20000)
        log(f"[bench] {coarse}^3 Newton at Re {re:g}: |P R(U)| {hist[-1]:.1e} ({time.perf_counter() - t0:.0f} s)")
    Uc = cc.get_base_flow().cpu().numpy()
    Uf = prolongate_velocity(Uc, cc.get_grid(), ctx.get_grid())
    cc.close()
    U, _, _ = ctx.project(torch.from_numpy(Uf).cuda(), tol=1e-12, max_iter=4)
    ctx.set_base_flow(U)
    ctx.set_stokes_precond(float("inf"))
    hist = []
    for step in range(9):
        _, r = ctx.newton_residual()
        hist.append(r)
        log(f"[bench] {ctx.nx}^3 Newton from the prolongated state, step {step}: |P R(U)| {r:.1e} "
            f"({time.perf_counter() - t0:.0f} s)")
        if r <= 1e-10 or step == 8:
            break
        ctx.newton_step(lin_tol=1e-8, gmres_m=100, max_vectors=6000)
    ctx.set_stokes_precond(0.0)
    return ctx.get_base_flow(), {"kind": "Newton steady state", "coarse_grid": coarse,
                                 "newton_res_inf": hist, "seconds": time.perf_counter() - t0}


def time_form(ctx, torch, inputs, warmup, steps, precision):
    vo = ctx.vel()
    po = ctx.cells()
    for q in range(warmup):
        ctx.krylov_vector(inputs[q % len(inputs)], vo, po, precision=precision, tol=1e-8)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for q in range(steps):
        _, _, st = ctx.krylov_vector(inputs[warmup + q], vo, po, precision=precision, tol=1e-8)
        if not st["converged"]:
            raise RuntimeError(f"step {q} did not converge: {st}")
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, stats


def train_guess(lk, torch, n, steps):
    """The learned guess, trained on an n^3 tanh-10 grid at the same Re (seeded
    synthetic base flow; pairs = the method's first SIMPLE corrections)."""
    tctx = lk.Context(n, n, n)
    tctx.set_stretching("tanh", TANH_RATIO)
    tctx.set_re(RE)
    tctx.set_lid(0.0)
    tctx.set_base_flow(synthetic_base_flow(tctx, torch))
    net = lk.Net(seed=11)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train(tctx, steps=steps, lr=2e-3, seed=7)
    dt = time.perf_counter() - t0
    tctx.close()
    return net, {"train_grid": f"{n}^3 tanh-10", "steps": steps, "seconds": dt,
                 "loss_first10": float(sum(hist[:10]) / max(1, min(10, steps))),
                 "loss_last30": float(sum(hist[-30:]) / max(1, min(30, steps)))}


def transform_flops(n, lines, symmetric):
    """FLOPs of one line transform of `lines` lines of length n: a dense n x n product,
    or on a mirror-symmetric axis the two half-size products (forward: he^2 + ho^2 per
    line; backward: he (he + ho)), averaged over the forward and backward launch."""
    if not symmetric:
        return 2.0 * n * n * lines
    he, ho = (n + 1) // 2, n // 2
    return 2.0 * lines * 0.5 * ((he * he + ho * ho) + he * (he + ho))


def kernel_table(prof, n, symmetric=True):
    """Per-kernel average durations and algorithmic rates (algorithmic bytes or FLOPs per
    launch over the launch's average HIP-event time)."""
    nx = ny = nz = n
    ncell = nx * ny * nz
    fu = 8.0 * ((nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1))  # bytes of a velocity
    fp = 8.0 * ncell
    alg = {
        "momentum": ("hbm", 3 * fu),             # read U, v; write w
        "divergence": ("hbm", fu + fp),          # read v; write r
        "correct": ("hbm", 2 * fu + 2 * fp),     # read w, phi; write v, p
        "tp_x": ("alu", transform_flops(nx, ny * nz, symmetric)),
        "tp_y": ("alu", transform_flops(ny, nx * nz, symmetric)),
        "tp_z": ("alu", transform_flops(nz, nx * ny, symmetric)),
        "eigscale": ("hbm", 2 * fp),
        "tridiag": ("hbm", 2 * fp),              # TPT: read the transformed field, write phi-hat
    }
    table = {}
    for name, (ms, launches) in prof.items():
        avg = ms / launches
        row = {"avg_ms": avg, "launches": launches, "total_ms": ms}
        if name in alg:
            kind, amount = alg[name]
            if kind == "hbm":
                row["GB/s"] = amount / (avg * 1e-3) / 1e9
                row["frac_hbm"] = row["GB/s"] / PEAK_HBM_GBS
            else:
                row["TFLOP/s"] = amount / (avg * 1e-3) / 1e12
                row["frac_fp64"] = row["TFLOP/s"] / PEAK_FP64_TFLOPS
            row["algorithmic"] = amount
        table[name] = row
    return table


def profile_traffic(cls, n):
    """HBM bytes per launch of a kernel class (FETCH_SIZE + WRITE_SIZE, calibrated) from
    the committed rocprofv3 summary of this workload, or None if the kernel's source
    file has changed since the counters were taken (or the workload differs)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"krylov_vector_{n}cubed_tanh10.txt")
    if not os.path.exists(path):
        return None
    for line in open(path).read().splitlines():
        p = line.split()
        if len(p) == 6 and p[0] == "traffic" and p[1] == cls:
            src = os.path.join(ROOT, p[4])
            if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != p[5]:
                return None
            return int(p[2]) + int(p[3])
    return None


def time_arnoldi(ctx, lk, torch, m=30, k=6):
    """Arnoldi extension steps (Krylov vector + FP64 Gram-Schmidt) per second:
    one implicitly restarted Arnoldi cycle (m vectors, one restart) on the benchmark
    context; convergence is not the point here."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.arnoldi_leading(k=k, m=m, tol=1e-12, max_restarts=1, seed=1, precision=lk.FP64, proj_tol=1e-8)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nvec = res["n_vectors"]
    return {"m": m, "k": k, "restarts": 1, "vectors": nvec, "seconds": dt, "steps_per_s": nvec / dt}


def cpu_baseline(n, reps=3):
    """The oracle (numpy/scipy, float64) on the host cores: Krylov vectors/s at n^3 and at
    100^3 (one warm-up, then the median of `reps` timed vectors each), and the first
    workload end to end at 16^3 (oracle Newton from rest to 1e-10, then ARPACK with 20
    vectors for the 4 leading eigenvalues)."""
    import statistics
    import numpy as np
    import synth
    from oracle import eigen, simple
    from oracle.grid import Grid
    from oracle.newton import Newton
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()

    def vectors_per_s(m):
        g = Grid.make(m, kind="tanh", ratio=TANH_RATIO)
        P = simple.Projector(g)
        U, _ = P.project(synth.random_velocity(m, m, m, 1000))
        U /= np.max(np.abs(U))
        times = []
        for s in range(reps + 1):               # the first is the warm-up
            v = synth.random_velocity(m, m, m, s + 1)
            t0 = time.perf_counter()
            P.krylov_vector(U, v, RE)
            if s:
                times.append(time.perf_counter() - t0)
        return 1.0 / statistics.median(times), times

    value, times = vectors_per_s(n)
    out = {"value": value, "unit": "Krylov vectors/s", "cores": threads, "kind": "oracle",
           "sample": f"1 warm-up + median of {reps} Krylov vectors at {n}^3 tanh-10, Re={RE:g} (numpy float64; "
                     f"stencils single-threaded, transforms on {threads} BLAS threads)",
           "seconds": times}
    if n != 100:
        v100, t100 = vectors_per_s(100)
        out["at_100"] = {"value": v100, "unit": "Krylov vectors/s", "seconds": t100}
    g = Grid.make(16)
    t0 = time.perf_counter()
    U, hist = Newton(g, 100.0, 0.0).solve(tol=1e-10)
    t1 = time.perf_counter()
    lam = eigen.arpack(g, U, 100.0, k=4, ncv=20, tol=1e-10)
    t2 = time.perf_counter()
    out["first_workload_16"] = {"newton_s": t1 - t0, "newton_steps": len(hist) - 1, "arnoldi_s": t2 - t1,
                                "total_s": t2 - t0, "leading": [[float(z.real), float(z.imag)] for z in lam[:4]],
                                "what": "16^3 uniform, Re=100, alpha=0: Newton (sparse direct) to |F| <= 1e-10, "
                                        "then ARPACK (20 vectors) for 4 leading eigenvalues"}
    return out


# Table 3 of the paper (sine grid of eq. 5): critical Re and frequency per grid, for the lid
# parallel to a side wall (alpha = 0) and to the diagonal plane (alpha = 45 degrees), and the
# grid-converged Richardson values
PAPER_TABLE3 = {0.0: {100: (1963.74, 0.575370), 150: (1938.98, 0.581315), 200: (1930.40, 0.583398),
                      256: (1926.10, 0.584438), "extrapolated": (1919.37, 0.58607)},
                45.0: {100: (2266.29, 0.250855), 150: (2278.39, 0.250305), 200: (2283.17, 0.249868),
                       256: (2285.56, 0.249650), "extrapolated": (2289.31, 0.249307)}}
# grids above 150^3 take the continuation path on the 100^3 grid and start from its steady state
CRITICAL_COARSE = 100
# per lid angle: the Newton continuation path from rest and, per grid, the two starting values
# of the secant search (alpha = 0: bracketing the paper's values on 100^3 - 256^3, at 200^3
# around the value an O(h^2) error predicts from this build's 100^3 and 150^3 results; alpha = 45:
# around the paper's 100^3 value, and at 150^3 around the value an O(h^2) error would give
# between the 100^3 result of this discretization, 2332.2, and the paper's limit, 2289.3)
CRITICAL_PATH = {0.0: ((250.0, 500.0, 800.0, 1100.0, 1400.0, 1600.0, 1750.0, 1850.0, 1900.0),
                       {"default": (1920.0, 1960.0), 200: (1928.0, 1935.0)}),
                 45.0: ((250.0, 500.0, 800.0, 1100.0, 1400.0, 1700.0, 1900.0, 2050.0, 2150.0, 2250.0),
                        {"default": (2265.0, 2285.0), 150: (2300.0, 2316.0)})}


# algorithmic HBM bytes per cell of the plane kernels of one projection with its potential:
# right side (two components in, one cell value out: 24), mode-space scaling (16; on the
# TPT route only the y-z planes take it, the planes containing x solve by the tridiagonal
# pass instead), correction (two components and phi in, three components out: 48), prefix
# sums (16)
PLANE_BYTES_PER_CELL = 24.0 + 16.0 + 48.0 + 16.0
PLANE_BYTES_PER_CELL_TPT = (2 * (PLANE_BYTES_PER_CELL - 16.0) + PLANE_BYTES_PER_CELL) / 3.0


def time_planes(ctx, torch, v, steps=10, route="tpt"):
    """Plane projections v1, v2, v3 with their potentials (eqs. 11-17) of one input:
    per family the mean wall time of a call (stream synchronized per call), then the
    per-class HIP-event times of one profiled pass over the three families."""
    n3 = ctx.nx * ctx.ny * ctx.nz
    out = ctx.vel()
    res = {}
    for which in (1, 2, 3):
        psi = torch.zeros(ctx.psi_size(which), dtype=torch.float64, device="cuda")
        ctx.plane_project(v, which, out, psi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.plane_project(v, which, out, psi)
        torch.cuda.synchronize()
        res[f"v{which}"] = {"ms_per_call": 1e3 * (time.perf_counter() - t0) / steps}
    ctx.profile(True)
    for _ in range(steps):
        for which in (1, 2, 3):
            psi = torch.zeros(ctx.psi_size(which), dtype=torch.float64, device="cuda")
            ctx.plane_project(v, which, out, psi)
    prof = ctx.profile_read()
    ctx.profile(False)
    calls = 3 * steps
    total = sum(ms for ms, _ in prof.values())
    res["projections_per_s_gpu_time"] = calls / (total * 1e-3)
    res["gpu_ms_per_projection"] = total / calls
    res["classes_ms_per_projection"] = {k: ms / calls for k, (ms, _) in prof.items()}
    if "planes" in prof:
        ms = prof["planes"][0] / calls
        per_cell = PLANE_BYTES_PER_CELL_TPT if route == "tpt" else PLANE_BYTES_PER_CELL
        gbs = per_cell * n3 / (ms * 1e-3) / 1e9
        res["plane_kernels"] = {"ms_per_projection": ms, "algorithmic_bytes": per_cell * n3,
                                "GB/s": gbs, "frac_hbm": gbs / PEAK_HBM_GBS}
    return res


def planes_run(n, lk, torch, steps, route):
    import synth
    ctx = lk.Context(n, n, n)
    ctx.set_stretching("tanh", TANH_RATIO)
    ctx.set_poisson_method(route)
    v = torch.from_numpy(synth.random_velocity(n, n, n, 1)).cuda()
    log(f"[planes] {n}^3 tanh-{TANH_RATIO:g}: {steps} calls per family")
    res = time_planes(ctx, torch, v, steps, route)
    res = {"metric": "plane projections with potentials (eqs. 11-17) per second", "grid": [n, n, n],
           "stretching": "tanh", "ratio": TANH_RATIO, **res}
    print(json.dumps(res), flush=True)


def critical_one(n, lk, torch, alpha_deg=0.0):
    """One grid: steady states continued from rest with Stokes-preconditioned Newton along
    the lid angle's path (up to Re 1900 for alpha = 0, 2250 for 45 degrees), then the secant
    search for the critical Reynolds number (the leading eigenvalue of eq. 7 crossing the
    imaginary axis) from the path's two starting values."""
    import math
    path, starts = CRITICAL_PATH[alpha_deg]
    re0, re1 = starts.get(n, starts["default"])
    t0 = time.perf_counter()
    cont = []
    vectors = 0

    def newton_at(c, tag, re):
        nonlocal vectors
        c.set_re(re)
        for step in range(12):
            _, r = c.newton_residual()
            log(f"[critical {tag}] Re {re:g} Newton step {step}: |P R(U)| {r:.2e} ({time.perf_counter() - t0:.0f} s)")
            if r <= 1e-11 or step == 11:
                break
            vectors += c.newton_step(lin_tol=1e-8, gmres_m=100, max_vectors=20000)["n_vectors"]
        cont.append({"grid": c.nx, "re": re, "newton_steps": step, "res_inf": r})

    def start(m):
        c = lk.Context(m)
        c.set_stretching("sine", 0.0)
        c.set_lid(math.radians(alpha_deg))
        c.set_base_flow(torch.zeros(c.nvel, dtype=torch.float64, device="cuda"))
        c.set_stokes_precond(float("inf"))
        return c

    ctx = start(n)
    if n > 150:
        # continuation on the coarse grid, then its steady state interpolated to this grid,
        # projected, and Newton here at the path's last Re
        cc = start(CRITICAL_COARSE)
        for re in path:
            newton_at(cc, CRITICAL_COARSE, re)
        Uf = prolongate_velocity(cc.get_base_flow().cpu().numpy(), cc.get_grid(), ctx.get_grid())
        cc.close()
        U, _, _ = ctx.project(torch.from_numpy(Uf).cuda(), tol=1e-12, max_iter=4)
        ctx.set_base_flow(U)
        newton_at(ctx, n, path[-1])
    else:
        for re in path:
            newton_at(ctx, n, re)
    t1 = time.perf_counter()
    os.environ["LK_VERBOSE"] = "1"  # progress trace on stderr during the long driver call
    out = ctx.critical_re(re0, re1, re_tol=1e-6, max_evals=8, newton_tol=1e-11, newton_steps=8,
                          lin_tol=1e-8, gmres_m=100, max_vectors=20000, k=8, m=100, eig_tol=1e-8,
                          max_restarts=150, seed=1, warm_start=True)
    os.environ["LK_VERBOSE"] = "0"
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.close()
    res = {"grid": [n, n, n], "re_cr": out["re_cr"], "omega_cr": out["omega_cr"], "converged": out["converged"],
           "evaluations": [{"re": h[0], "re_lambda": h[1], "im_lambda": h[2], "res_inf": h[3]}
                           for h in out["history"]],
           "continuation": cont, "continuation_krylov_vectors": vectors,
           "seconds_continuation": t1 - t0, "seconds_critical": t2 - t1}
    if n in PAPER_TABLE3[alpha_deg]:
        pre, pom = PAPER_TABLE3[alpha_deg][n]
        res["paper_table3"] = {"re_cr": pre, "omega_cr": pom, "re_rel_diff": out["re_cr"] / pre - 1.0,
                               "omega_rel_diff": out["omega_cr"] / pom - 1.0}
    return res


def richardson(v_coarse, v_fine, n_coarse, n_fine):
    """Richardson extrapolation of a value with an O(h^2) error, h = 1/n (Section 5)."""
    return v_fine + (v_fine - v_coarse) / ((n_fine / n_coarse) ** 2 - 1.0)


def critical_run(sizes, lk, torch, alpha_deg=0.0):
    """Critical Reynolds number on each grid of the sequence (sine grid of eq. 5, lid at
    angle alpha to x) and the Richardson extrapolation of Section 5 from each pair of
    consecutive grids: with an O(h^2) error, v = v_f + (v_f - v_c) / ((n_f / n_c)^2 - 1)."""
    grids = [critical_one(n, lk, torch, alpha_deg) for n in sizes]
    extrap = []
    for c, f in zip(grids, grids[1:]):
        nc, nf = c["grid"][0], f["grid"][0]
        extrap.append({"grids": [nc, nf], "re_cr": richardson(c["re_cr"], f["re_cr"], nc, nf),
                       "omega_cr": richardson(c["omega_cr"], f["omega_cr"], nc, nf)})
    res = {"metric": "critical Reynolds number (leading eigenvalue of eq. 7 crossing the imaginary axis)",
           "stretching": "sine (eq. 5)", "alpha_deg": alpha_deg, "newton": "Stokes-preconditioned (dt = inf)",
           "grids": grids, "richardson": extrap,
           "paper_table3_extrapolated": dict(zip(("re_cr", "omega_cr"), PAPER_TABLE3[alpha_deg]["extrapolated"]))}
    print(json.dumps(res), flush=True)


def steady_states(lk, torch, n, alpha_deg, res_wanted):
    """Newton steady states of the n^3 tanh-10 cube at each Re of res_wanted (continued from
    rest, Stokes-preconditioned Newton to max |P R(U)| <= 1e-10; a state that stops short of
    that but below 1e-6 is kept for training, its residual recorded); returns
    {Re: (U, max |P R(U)|)}."""
    import math
    ctx = lk.Context(n)
    ctx.set_stretching("tanh", TANH_RATIO)
    ctx.set_lid(math.radians(alpha_deg))
    ctx.set_base_flow(torch.zeros(ctx.nvel, dtype=torch.float64, device="cuda"))
    ctx.set_stokes_precond(float("inf"))
    out = {}
    path = sorted(set([250.0 * q for q in range(1, 9)] + [2000.0 + 125.0 * q for q in range(1, 5)] +
                      [r for r in res_wanted]))
    for re in path:
        ctx.set_re(re)
        hist = ctx.newton(tol=1e-10, max_steps=15, lin_tol=1e-9, gmres_m=100, max_vectors=20000)
        log(f"[recipe] {n}^3 alpha {alpha_deg:g} Re {re:g}: Newton |P R(U)| {hist[-1]:.1e} ({len(hist) - 1} steps)")
        if not hist[-1] <= 1e-6:
            raise RuntimeError(f"Newton did not converge at {n}^3, alpha {alpha_deg}, Re {re}")
        if re in res_wanted:
            out[re] = (ctx.get_base_flow().clone(), hist[-1])
    ctx.close()
    return out


def learned_recipe_run(lk, torch, pairs, rounds, save_net=""):
    """The learned guess trained on the training set of the learned-preconditioner workload:
    pairs the method generates (w = L_U v, D w -> the first SIMPLE correction) on 64^3 and
    100^3 tanh-10 grids, on Newton steady states at Re 1000..2500 for both lid directions
    (parallel to a side wall, alpha = 0, and to the diagonal plane, alpha = 45 degrees),
    visited round-robin; then evaluated inside SIMPLE at 150^3 and 200^3 (the benchmark's
    Re = 1900 and seeded base flow) and at 150^3 on the Newton steady state at Re = 1900,
    against the same network after 300 64^3 pairs and an untrained one.  save_net: file the
    trained parameters are written to right after training.  One JSON line."""
    import math
    t0 = time.perf_counter()
    spec = {64: (1000.0, 1500.0, 2000.0, 2500.0), 100: (1000.0, 1750.0, 2500.0)}
    states = []  # (n, alpha, Re, U)
    residuals = []
    for n, res in spec.items():
        for alpha in (0.0, 45.0):
            for re, (U, r) in steady_states(lk, torch, n, alpha, res).items():
                states.append((n, alpha, re, U))
                residuals.append({"grid": n, "alpha_deg": alpha, "re": re, "res_inf": r})
    t1 = time.perf_counter()
    ctxs = {}
    for n in spec:
        c = lk.Context(n)
        c.set_stretching("tanh", TANH_RATIO)
        ctxs[n] = c
    net = lk.Net(seed=11)
    per = max(1, pairs // (rounds * len(states)))
    losses = []
    for rnd in range(rounds):
        lr = 2e-3 if rnd < rounds // 2 else (1e-3 if rnd < 3 * rounds // 4 else 5e-4)
        for q, (n, alpha, re, U) in enumerate(states):
            c = ctxs[n]
            c.set_re(re)
            c.set_lid(math.radians(alpha))
            c.set_base_flow(U)
            h = net.train(c, steps=per, lr=lr, seed=1 + rnd * len(states) + q)
            losses.append(float(h.mean()))
        log(f"[recipe] round {rnd}: mean loss {sum(losses[-len(states):]) / len(states):.4f} "
            f"({time.perf_counter() - t1:.0f} s)")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if save_net:
        net.save(save_net)
    for c in ctxs.values():
        c.close()
    quick, _ = train_guess(lk, torch, 64, 300)
    untrained = lk.Net(seed=11)
    evals = []
    for n, base in ((150, "seeded"), (200, "seeded"), (150, "steady")):
        ctx = lk.Context(n)
        ctx.set_stretching("tanh", TANH_RATIO)
        ctx.set_lid(0.0)
        if base == "seeded":
            ctx.set_re(RE)
            ctx.set_base_flow(synthetic_base_flow(ctx, torch))
        else:
            ctx.set_base_flow(torch.zeros(ctx.nvel, dtype=torch.float64, device="cuda"))
            ctx.set_stokes_precond(float("inf"))
            for re in (500.0, 1000.0, 1500.0, RE):
                ctx.set_re(re)
                hist = ctx.newton(tol=1e-10, max_steps=15, lin_tol=1e-9, gmres_m=100, max_vectors=20000)
                log(f"[recipe] {n}^3 steady state, Re {re:g}: Newton |P R(U)| {hist[-1]:.1e} ({len(hist) - 1} steps)")
            ctx.set_stokes_precond(0.0)
        inputs = make_inputs(ctx, torch, 8, seed0=901)
        row = {"grid": [n, n, n], "base_flow": base}
        for name, nt in (("recipe", net), ("bench_300", quick), ("untrained", untrained)):
            ctx.set_net(nt)
            dt, stats = time_form(ctx, torch, inputs, 2, 6, lk.LEARNED)
            row[name] = {"guess_eps_mean": sum(st["guess_eps"] for st in stats) / len(stats),
                         "rho_first_pass_mean": sum(st["rho_hist"][0] for st in stats) / len(stats),
                         "passes_mean": sum(st["iterations"] for st in stats) / len(stats),
                         "vectors_per_s": 6 / dt}
        dt, stats = time_form(ctx, torch, inputs, 2, 6, lk.MIXED)
        row["mixed"] = {"rho_first_pass_mean": sum(st["rho_hist"][0] for st in stats) / len(stats),
                        "passes_mean": sum(st["iterations"] for st in stats) / len(stats), "vectors_per_s": 6 / dt}
        log(f"[recipe] {n}^3 {base}: eps recipe {row['recipe']['guess_eps_mean']:.3f}, 300-pair "
            f"{row['bench_300']['guess_eps_mean']:.3f}, untrained {row['untrained']['guess_eps_mean']:.3f}")
        evals.append(row)
        ctx.close()
    res = {"metric": "learned guess: continuity residual after the guess relative to a plain start (eps)",
           "training_set": {"grids": ["64^3 tanh-10", "100^3 tanh-10"], "re": {str(k): v for k, v in spec.items()},
                            "alpha_deg": [0.0, 45.0], "base_flows": "Newton steady states",
                            "newton_residuals": residuals,
                            "pairs": per * rounds * len(states), "rounds": rounds, "pairs_per_visit": per,
                            "seconds_newton": t1 - t0, "seconds_training": t2 - t1,
                            "loss_first_round": sum(losses[:len(states)]) / len(states),
                            "loss_last_round": sum(losses[-len(states):]) / len(states)},
           "evaluation": evals}
    print(json.dumps(res), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the multi-GPU layout is a design note, not a build)", file=sys.stderr)
        sys.exit(1)
    import torch
    import paper_1704_08521_amd as lk
    if a.critical:
        torch.cuda.set_device(0)
        critical_run([int(x) for x in a.critical.split(",")], lk, torch, a.alpha)
        return
    if a.planes:
        torch.cuda.set_device(0)
        planes_run(a.size, lk, torch, a.steps, a.poisson)
        return
    if a.learned_recipe:
        torch.cuda.set_device(0)
        learned_recipe_run(lk, torch, a.learned_recipe, rounds=10, save_net=a.save_net)
        return
    n = a.size
    torch.cuda.set_device(0)
    ctx = lk.Context(n, n, n)
    ctx.set_stretching("tanh", TANH_RATIO)
    ctx.set_re(RE)
    ctx.set_lid(0.0)
    ctx.set_poisson_method(a.poisson)
    log(f"[bench] {n}^3 tanh-{TANH_RATIO:g} Re={RE:g}: building inputs")
    if a.base_flow == "steady":
        U, base_info = steady_base_flow(lk, torch, ctx)
    else:
        U = synthetic_base_flow(ctx, torch)
        base_info = {"kind": "seeded divergence-free field, max |U| = 1"}
    ctx.set_base_flow(U)
    inputs = make_inputs(ctx, torch, a.warmup + a.steps)
    # the streaming ceiling of this device for the stencil's pattern (2 reads + 1 write) and
    # for a copy: plain 16-byte-access kernels over velocity-sized arrays
    import ctypes
    lib = lk._lib.load()
    ceiling = {}
    for kind, name in ((1, "read2_write1"), (0, "copy"), (2, "read")):
        tb, us = ctypes.c_double(), ctypes.c_double()
        rc = lib.lc_stream_probe(kind, ctypes.c_size_t(8 * ctx.nvel), 20, ctypes.c_void_p(
            torch.cuda.current_stream().cuda_stream), ctypes.byref(tb), ctypes.byref(us))
        if rc == 0:
            ceiling[name] = {"TB/s": tb.value, "us": us.value, "frac_of_peak": tb.value * 1e3 / PEAK_HBM_GBS}
    log(f"[bench] streaming ceiling: " + ", ".join(f"{k} {v['TB/s']:.2f} TB/s" for k, v in ceiling.items()))
    # calibration for hardware byte counters: one plain device copy of 256 MiB
    calib = torch.empty(1 << 25, dtype=torch.float64, device="cuda")
    calib.copy_(inputs[0][: 1].expand(1 << 25))
    torch.empty_like(calib).copy_(calib)
    del calib
    torch.cuda.synchronize()

    log(f"[bench] training the learned guess: {a.train_steps} steps on {a.train_size}^3")
    net, training = train_guess(lk, torch, a.train_size, a.train_steps)
    ctx.set_net(net)
    log(f"[bench] trained in {training['seconds']:.1f} s, loss {training['loss_first10']:.3f} -> "
        f"{training['loss_last30']:.3f}")

    forms = {}
    outs = {}
    for name, prec in (("plain", lk.FP64), ("mixed", lk.MIXED), ("learned", lk.LEARNED)):
        dt, stats = time_form(ctx, torch, inputs, a.warmup, a.steps, prec)
        iters = [st["iterations"] for st in stats]
        forms[name] = {"value": a.steps / dt, "ms_per_step": 1e3 * dt / a.steps,
                       "simple_passes_mean": sum(iters) / len(iters),
                       "rho_first_pass_mean": sum(st["rho_hist"][0] for st in stats) / len(stats)}
        if name == "learned":
            forms[name]["guess_used"] = sum(st["guess_used"] for st in stats)
            forms[name]["guess_eps_mean"] = sum(st["guess_eps"] for st in stats) / len(stats)
            forms[name]["training"] = training
            forms[name]["passes"] = "mixed"
        outs[name], _, _ = ctx.krylov_vector(inputs[0], precision=prec, tol=1e-8)
        log(f"[bench] {name}: {forms[name]['value']:.1f} vectors/s, {forms[name]['ms_per_step']:.3f} ms/step, "
            f"passes {forms[name]['simple_passes_mean']:.2f}")
    ref = outs["plain"]
    for name in ("mixed", "learned"):
        forms[name]["rel_diff_vs_plain"] = float(torch.linalg.vector_norm(outs[name] - ref) /
                                                 torch.linalg.vector_norm(ref))
        # the measured quantity of each form against plain: time per vector (> 1: slower)
        forms[name]["time_vs_plain"] = forms[name]["ms_per_step"] / forms["plain"]["ms_per_step"]

    # profiled repeat of the plain timed loop: per-kernel HIP events on the context stream
    ctx.profile(True)
    time_form(ctx, torch, inputs, 0, a.steps, lk.FP64)
    prof = ctx.profile_read()
    ctx.profile(False)
    table = kernel_table(prof, n, symmetric=True)  # the tanh grid is mirror-symmetric
    # the learned form's network forward pass (all layers), same method
    ctx.profile(True)
    time_form(ctx, torch, inputs, 0, min(a.steps, 5), lk.LEARNED)
    lprof = ctx.profile_read()
    ctx.profile(False)
    if "nn_forward" in lprof:
        ms, launches = lprof["nn_forward"]
        avg = ms / launches
        flops = NN_FLOP_PER_VOXEL * (((n + 3) // 4 * 4) ** 3)
        forms["learned"]["nn_forward"] = {"avg_ms": avg, "launches": launches, "TFLOP/s": flops / (avg * 1e-3) / 1e12,
                                          "frac_bf16_mfma": flops / (avg * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
                                          "algorithmic_flop": flops}
    dom = max((k for k in table if "algorithmic" in table[k]), key=lambda k: table[k]["total_ms"])
    d = table[dom]
    if "TFLOP/s" in d:
        # the symmetric-grid transforms run on the FP64 matrix cores (same 78.6 TFLOP/s peak)
        roof = {"bound": "mfma", "achieved": d["TFLOP/s"], "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": d["frac_fp64"], "traffic": profile_traffic(dom, n), "kernel": dom, "avg_ms": d["avg_ms"]}
    else:
        roof = {"bound": "hbm", "achieved": d["GB/s"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": d["frac_hbm"], "traffic": profile_traffic(dom, n), "kernel": dom, "avg_ms": d["avg_ms"]}
    for name, row in table.items():
        t = profile_traffic(name, n)
        if t is not None:
            row["traffic"] = t
    if roof["bound"] == "hbm" and "read2_write1" in ceiling:
        # the same kernel against what a plain kernel with its access pattern reaches here
        roof["ceiling"] = ceiling["read2_write1"]["TB/s"] * 1e3
        roof["frac_of_ceiling"] = roof["achieved"] / roof["ceiling"]

    log("[bench] Arnoldi cycle (m=30, k=6, one restart)")
    arnoldi = time_arnoldi(ctx, lk, torch)
    log(f"[bench] Arnoldi: {arnoldi['steps_per_s']:.1f} steps/s ({arnoldi['vectors']} vectors)")
    planes = time_planes(ctx, torch, inputs[0], route=a.poisson)
    log(f"[bench] plane projections: {planes['gpu_ms_per_projection']:.3f} ms GPU time each")
    out = {
        "metric": "Krylov vectors/s to 1e-8 rel. residual at 200^3 (plain/mixed/learned); % HBM peak",
        "value": forms["plain"]["value"],
        "unit": "Krylov vectors/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": forms["plain"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"krylov_vector {n}^3 tanh-10 stretched, Re={RE:g}, alpha=0, rho<=1e-8, "
                               "seeded projected random inputs, base flow: " + base_info["kind"],
                   "base_flow": base_info,
                   "grid": [n, n, n], "stretching": "tanh", "ratio": TANH_RATIO, "re": RE, "tol": 1e-8,
                   "poisson": "tensor-product factorization"},
        "forms": forms,
        "arnoldi": arnoldi,
        "planes": planes,
        "roofline": roof,
        "stream_ceiling": ceiling,
        "kernels": table,
    }
    if not a.no_cpu:
        log(f"[bench] cpu baseline: oracle Krylov vectors at {n}^3 and 100^3, first workload at 16^3")
        out["cpu_baseline"] = cpu_baseline(n, a.cpu_reps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
