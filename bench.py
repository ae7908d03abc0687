#!/usr/bin/env python3
"""Benchmark of the treecode Green-function convolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload atom|cube]

A step is one pass of the whole path on the workload: tree build and batches,
upward pass, interaction lists and schedule, far and near fields, combine, for
every convolution the workload holds. The default workload is the single-atom
adaptive mesh (Be-like Z = 4 in [-20, 20]^3, 1,007,616 Fejer points): a Yukawa
convolution (kappa = sqrt(0.4)) of psi_1s + psi_2s and a Coulomb (Hartree)
convolution of rho = 2 psi_1s^2 + 2 psi_2s^2, both singularity-subtracted, on one
tree with N_L = 2000, each at the cheapest (theta, degree) found that holds it to
1e-6 (Yukawa 0.75, 8; Coulomb 0.8, 8); the accuracy of theta = 0.8, degree 8,
N_L = 500 is reported beside it.
Inputs are resident in HBM before timing.

Printed: one JSON line with the throughput (batch-cluster kernel evaluations
per second, far + near, over the whole step), the accuracy against the GPU
direct sum on sampled targets, the roofline position of the dominant kernel
(the interaction kernel, timed with HIP events on its own stream; its HBM
traffic comes from the FETCH_SIZE / WRITE_SIZE counter profile committed under
profiles/, reported only while the kernel sources match the profiled ones) and
the CPU oracle's rate on a bounded sample. Unless --no-compare is given, it also
holds two comparisons: Lagrange against Hermite interpolation on the atom at
the accuracy targets 1e-6 and 1e-9, and the plain, batched, mixed-precision and
learned-selector variants on the 21 benzene orbitals (with the GPU mesh build).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Green-convolution time & interactions/s at 1e-6 rel err; batched/mixed vs plain"
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector peak

# Algorithmic FP64 flops per kernel evaluation (FMA = 2): squared distance (8
# for particle sources; 3 for proxy sources, whose tensor grid gives d^2 with one
# subtraction and one multiply-add per pair), reciprocal square root (seed plus
# one Newton step, 7; 9 when the same step also gives d), exp as a power of two
# whose reduced argument comes from the scaled decay constant in one multiply-add,
# and a degree-9 polynomial (24), the products forming the kernel value, and two
# multiply-adds (4). The far field of the Gaussian-subtracted
# Coulomb kernel takes the Gaussian as the product of per-dimension factors: two
# multiplies per evaluation, and 3 (n+1) exponentials per target and cluster
# that are not counted.
FLOPS = {
    ("yukawa_ss", "far"): 3 + 9 + 24 + 1 + 4,
    ("yukawa_ss", "near"): 8 + 9 + 24 + 1 + 4,
    ("coulomb_ss", "far"): 3 + 7 + 2 + 4,
    ("coulomb_ss", "near"): 8 + 7 + 24 + 1 + 2 + 2,
}


# Coulomb-SS pairs between boxes at least 6.12 alpha apart skip the Gaussian
# term (its value is below 2^-54): a near evaluation is then squared distance (8),
# reciprocal square root (7) and one multiply-add (2); a far one (blocks of up to
# 4 orbitals, FP64) squared distance (3), reciprocal square root (7) and one
# multiply-add (2)
COULOMB_NEAR_1R_FLOPS = 8 + 7 + 2
COULOMB_FAR_1R_FLOPS = 3 + 7 + 2
GAUSS_SKIP = 37.5  # (box gap / alpha)^2 above which the kernel skips the Gaussian


def coulomb_gauss_skipped(tagi, x, y, z, leaf, box, theta, degree, alpha=1.0):
    """(near, far) evaluations of a Coulomb-SS convolution that take the 1/d-only
    path: (batch, cluster) pairs whose boxes lie at least 6.12 alpha apart, by the
    kernel's own rule applied to the exported tree and lists."""
    t = tagi.Tree(x, y, z, leaf, box)
    e = t.export()
    L = t.lists(theta, degree)
    t.close()
    leaves = np.nonzero(e["n_child"] == 0)[0]
    cnt = (e["end"] - e["begin"]).astype(np.int64)

    def skipped(off, ids, per_cluster):
        B = np.repeat(leaves, np.diff(off))
        gap = np.maximum(0.0, np.maximum(e["lo"][ids] - e["hi"][B], e["lo"][B] - e["hi"][ids]))
        skip = (gap * gap).sum(axis=1) / (alpha * alpha) > GAUSS_SKIP
        return int((cnt[B] * per_cluster(ids))[skip].sum())

    near = skipped(L["near_off"], L["near_id"], lambda C: cnt[C])
    far = skipped(L["far_off"], L["far_id"], lambda C: np.int64((degree + 1) ** 3))
    return near, far


# counter profile of the interaction kernel and the sources it was taken from
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_interact_atom_mesh_Z4.md")
KERNEL_SOURCES = ["interact_impl.hpp", "devmath.hpp", "interact_yukawa_ss.hip",
                  "interact_coulomb_ss.hip", "interact.hip", "lists.hip"]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2003_01833_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def workload_key(config: dict) -> str:
    """One line naming the workload and every convolution's setting."""
    convs = " ".join(f"{k} theta {v['theta']} degree {v['degree']}"
                     for k, v in config["settings"].items())
    return f"{config['workload']} {convs} leaf {config['leaf_size']}"


def counter_traffic(config: dict):
    """HBM bytes per interaction-kernel launch (FETCH_SIZE and WRITE_SIZE, each
    scaled by its reading for a copy of known size) from the committed profile, or
    None when the profile is missing, was taken on another workload, or the kernel
    sources changed since."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            kv = dict(re.findall(r"^- `(\w+)`: `([^`]*)`", fh.read(), re.M))
    except OSError:
        return None
    want = workload_key(config)
    if kv.get("workload") != want or kv.get("source_sha256") != kernel_source_digest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def make_workload(name: str):
    from workloads.configs import DOMAIN, atom_mesh, uniform_cube
    if name == "atom":
        d = atom_mesh()
        # each convolution at the cheapest (theta, degree) of the parameter sweep
        # that meets 1e-6 relative L2 and max error on one tree (N_L = 2000); the
        # workload's stated setting (theta 0.8, degree 8, N_L 500) is run once for
        # its error
        convs = [dict(kernel="yukawa_ss", f=d["psi"], kappa=float(d["kappa"]), theta=0.75,
                      degree=8),
                 dict(kernel="coulomb_ss", f=d["rho"], kappa=0.0, theta=0.8, degree=8)]
        return dict(name="atom_mesh_Z4", x=d["x"], y=d["y"], z=d["z"], w=d["w"], convs=convs,
                    leaf=2000, stated=(0.8, 8, 500), box=(*DOMAIN[0], *DOMAIN[1]))
    x, y, z, f, w = uniform_cube(32768, seed=1)
    return dict(name="uniform_cube_32768", x=x, y=y, z=z, w=w,
                convs=[dict(kernel="yukawa_ss", f=f, kappa=1.0, theta=0.7, degree=6)],
                leaf=500, box=None)


def cpu_baseline(wl, seconds: float):
    """The oracle's direct sum on sampled targets (all sources), both kernels."""
    from oracle.direct import default_threads, direct_sum
    from workloads.configs import sample_targets
    threads = min(16, default_threads())
    n = wl["x"].size

    def run(k):
        idx = sample_targets(n, k, seed=4)
        t0 = time.perf_counter()
        for c in wl["convs"]:
            f = c["f"]
            direct_sum(c["kernel"], wl["x"], wl["y"], wl["z"], f, wl["w"], wl["x"][idx],
                       wl["y"][idx], wl["z"][idx], f[idx], kappa=c["kappa"] or 1.0,
                       threads=threads)
        return time.perf_counter() - t0

    probe = max(threads, 16)
    dt = run(probe)
    k = int(min(n, max(probe, probe * seconds / max(dt, 1e-6))))
    dt = run(k)
    pairs = k * n * len(wl["convs"])
    # one thread, for the per-core rate (a tenth of the time)
    k1 = max(1, int(k * 0.1 / max(threads, 1)))
    idx1 = sample_targets(n, k1, seed=5)
    t0 = time.perf_counter()
    for c in wl["convs"]:
        f = c["f"]
        direct_sum(c["kernel"], wl["x"], wl["y"], wl["z"], f, wl["w"], wl["x"][idx1],
                   wl["y"][idx1], wl["z"][idx1], f[idx1], kappa=c["kappa"] or 1.0, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"direct sum at {k} seeded targets x {n} sources for "
                      f"{len(wl['convs'])} kernel(s), {dt:.1f} s",
            # the full N^2 direct sums of one step at the sampled rate
            "extrapolated_full_direct_s": n * n * len(wl["convs"]) / (pairs / dt),
            "per_core_value": k1 * n * len(wl["convs"]) / dt1,
            "per_core_sample": f"{k1} targets on 1 thread, {dt1:.1f} s"}


def compare_batched(tagi, torch, fp64=(0.7, 8), mixed=(0.8, 10), leaf=2000, samples=10000,
                    reps=1):
    """The benzene workload (4,143,104 points, 21 orbitals, one kappa each): the
    per-orbital FP64 loop and one batched FP64 launch sequence at the cheapest
    FP64 (theta, degree) found that meets 1e-6, batched with the mixed-precision
    far field at the cheapest such setting for it, and the learned selector.
    Times exclude the tree build and include upward, lists (cached after the
    first call) and the convolution; errors are per orbital against the GPU
    direct sum at sampled targets."""
    theta, degree = fp64
    from workloads.configs import DOMAIN, benzene_mesh, benzene_orbitals, sample_targets
    _log("compare: building the benzene mesh and 21 orbitals")
    t0 = time.perf_counter()
    m = benzene_mesh()
    cpu_mesh_ms = 1e3 * (time.perf_counter() - t0)
    orb = benzene_orbitals(m["x"], m["y"], m["z"])
    n = m["x"].size
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    # the same mesh built on the GPU (adaptive refinement and the quadrature points)
    from workloads.configs import benzene_atoms
    atoms = [(tuple(R), Z) for R, Z in benzene_atoms()]
    gpu_mesh = lambda: tagi.mesh(DOMAIN[0], DOMAIN[1], 7, 5e-4, 4, atoms=atoms,  # noqa: E731
                                 test="root_density_vext")
    gpu_mesh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gx, gy, gz, gw, glo, _ = gpu_mesh()
    torch.cuda.synchronize()
    mesh_info = {"cells": int(glo.shape[0]), "points": int(gx.numel()),
                 "gpu_ms": 1e3 * (time.perf_counter() - t0),
                 "cpu_input_generator_ms": cpu_mesh_ms,
                 "same_points_as_cpu": bool(np.array_equal(gx.cpu().numpy(), m["x"]) and
                                            np.allclose(gw.cpu().numpy(), m["w"], rtol=1e-15,
                                                        atol=0))}
    del gx, gy, gz, gw
    x, y, z, w = dev(m["x"]), dev(m["y"]), dev(m["z"]), dev(m["w"])
    F = dev(orb["psi"])
    kap = orb["kappa"]
    n_orb = F.shape[0]
    t = tagi.Tree(x, y, z, leaf, (*DOMAIN[0], *DOMAIN[1]))
    idx = torch.from_numpy(sample_targets(n, samples, seed=4)).cuda()
    sub = lambda a: a[idx].contiguous()  # noqa: E731
    refs = [tagi.direct("yukawa_ss", x, y, z, F[o].contiguous(), w, sub(x), sub(y), sub(z),
                        sub(F[o]), kappa=float(kap[o])) for o in range(n_orb)]

    def errors(U):
        e = []
        for o in range(n_orb):
            u = U[o, idx]
            e.append((float(torch.linalg.norm(u - refs[o]) / torch.linalg.norm(refs[o])),
                      float((u - refs[o]).abs().max() / refs[o].abs().max())))
        return {"rel_l2_max_over_orbitals": max(a for a, _ in e),
                "rel_max_max_over_orbitals": max(b for _, b in e),
                "rel_l2_per_orbital": [a for a, _ in e],
                "rel_max_per_orbital": [b for _, b in e]}

    def timed(fn, warm=None):
        # warm: a cheaper call that prepares the same plans and lists (default: fn)
        (warm or fn)()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, 1e3 * (time.perf_counter() - t0) / reps

    U_plain = torch.empty((n_orb, n), dtype=torch.float64, device="cuda")

    def plain():
        for o in range(n_orb):
            t.upward(F[o].contiguous(), w, degree)
            t.convolve("yukawa_ss", float(kap[o]), theta, degree, out=U_plain[o:o + 1])
        return U_plain

    res = {"workload": "benzene_mesh_21_orbitals", "n_points": n, "n_orb": n_orb,
           "mesh_build": mesh_info,
           "leaf_size": leaf, "fp64_setting": {"theta": theta, "degree": degree},
           "mixed_setting": {"theta": mixed[0], "degree": mixed[1]}}
    _log("compare: plain per-orbital loop")
    def plain_warm():
        # one orbital prepares the lists and the single-orbital schedule and plan
        t.upward(F[0].contiguous(), w, degree)
        t.convolve("yukawa_ss", float(kap[0]), theta, degree, out=U_plain[0:1])

    U, ms = timed(plain, warm=plain_warm)
    res["plain_fp64"] = {"ms": ms, **errors(U)}

    def batched(precision, th, deg):
        def run():
            t.upward(F, w, deg)
            return t.convolve("yukawa_ss", kap, th, deg, precision=precision)
        return run

    _log("compare: batched FP64")
    U, ms = timed(batched("fp64", theta, degree))
    st = t.stats()
    res["batched_fp64"] = {"ms": ms, **errors(U),
                           "interactions_per_orbital": st["far_interactions"] + st["near_interactions"]}
    # the same step captured as a HIP graph (upward + convolve), replayed
    Ug = torch.empty((n_orb, n), dtype=torch.float64, device="cuda")
    g = t.graph(F, w, degree, "yukawa_ss", kap, theta, out=Ug)
    # creating the graph ran the step once: the plans are ready
    _, ms_g = timed(lambda: g.launch(), warm=lambda: None)
    res["batched_fp64"]["graph_replay_ms"] = ms_g
    res["batched_fp64"]["graph_equals_eager"] = bool(torch.equal(Ug, U))
    g.close()
    # autotuned leaf size and orbital block (timed on the first eight orbitals),
    # then the batched FP64 step with the pick on all orbitals
    _log("compare: autotuning N_L and the orbital block")
    cand_leaf, cand_ob = (2000, 4000), (4, 8)
    (leaf_t, ob_t), times = tagi.autotune(x, y, z, F[:8].contiguous(), w, "yukawa_ss", kap[:8],
                                          theta, degree, leaf_sizes=cand_leaf, obs=cand_ob,
                                          box=(*DOMAIN[0], *DOMAIN[1]))
    tt = t if leaf_t == leaf else tagi.Tree(x, y, z, leaf_t, (*DOMAIN[0], *DOMAIN[1]))
    tt.set_orbital_block(ob_t)

    def tuned():
        tt.upward(F, w, degree)
        return tt.convolve("yukawa_ss", kap, theta, degree)
    U, ms = timed(tuned)
    res["batched_fp64_autotuned"] = {
        "ms": ms, **errors(U), "leaf_size": leaf_t, "orbital_block": ob_t,
        "tuning_ms_per_step_8_orbitals": {f"N_L {a} OB {b}": float(times[i, j])
                                          for i, a in enumerate(cand_leaf)
                                          for j, b in enumerate(cand_ob)}}
    tt.set_orbital_block(0)
    if tt is not t:
        tt.close()
    _log("compare: batched mixed")
    U, ms = timed(batched("mixed", *mixed))
    st_m = t.stats()
    res["batched_mixed"] = {"ms": ms, **errors(U), "interactions_per_orbital":
                            st_m["far_interactions"] + st_m["near_interactions"]}
    weights = os.path.join(ROOT, "paper_2003_01833_amd", "selector_weights.npz")
    if os.path.exists(weights):
        from paper_2003_01833_amd.selector import Selector
        sel = Selector.load(weights)
        eta = float(sel.meta.get("eta", 0.01))
        # per-orbital pair budget from the FP64 result's magnitude (in a Green
        # iteration: the previous iterate's)
        U64 = batched("fp64", theta, degree)()
        tol = eta * 1e-6 * U64.abs().amax(dim=1).cpu().numpy()
        for prec in ("fp64", "mixed"):
            def learned(prec=prec):
                # the learned path forms its own per-degree proxy charges; the
                # upward pass only has to stage f and w (lowest degree)
                t.upward(F, w, 1)
                return t.convolve_learned("yukawa_ss", kap, sel, tol, precision=prec)
            _log(f"compare: batched {prec} + learned selector")
            t0 = time.perf_counter()
            learned()
            torch.cuda.synchronize()
            first_ms = 1e3 * (time.perf_counter() - t0)
            U, ms = timed(learned)
            ls = t.learned_stats()
            res[f"batched_{prec}_learned"] = {
                "ms": ms, "first_call_ms_with_lists": first_ms, "eta": eta, **errors(U),
                "interactions_per_orbital": ls["far_interactions"] + ls["near_interactions"],
                "far_pairs_by_degree": ls["far_pairs_by_degree"]}
    res["speedup_batched_vs_plain"] = res["plain_fp64"]["ms"] / res["batched_fp64"]["ms"]
    res["speedup_mixed_vs_plain"] = res["plain_fp64"]["ms"] / res["batched_mixed"]["ms"]
    res["speedup_autotuned_vs_plain"] = (res["plain_fp64"]["ms"] /
                                         res["batched_fp64_autotuned"]["ms"])
    if "batched_mixed_learned" in res:
        res["speedup_mixed_learned_vs_plain"] = (res["plain_fp64"]["ms"] /
                                                 res["batched_mixed_learned"]["ms"])
    t.close()
    return res


# Cheapest settings of each interpolation form (N_L = 2000, the tree of the timed
# step) reaching a maximum relative error of 1e-6 and of 1e-9 on the Be-like mesh,
# from parameter sweeps (Lagrange degrees 8-14, Hermite degrees 4-7, theta
# 0.5-0.9): (theta, degree).
HERMITE_COMPARE = {
    "yukawa_ss": {"1e-6": {"lagrange": (0.75, 8), "hermite": (0.8, 6)},
                  "1e-9": {"lagrange": (0.7, 12), "hermite": (0.5, 6)}},
    "coulomb_ss": {"1e-6": {"lagrange": (0.8, 8), "hermite": (0.8, 5)},
                   "1e-9": {"lagrange": (0.7, 11), "hermite": (0.5, 6)}},
}


def compare_hermite(tagi, torch, x, y, z, w, fields, refs, idx, leaf, box, reps=3):
    """Lagrange against Hermite interpolation at two accuracy targets: the median
    of `reps` convolutions after one warm-up, and the error at the sampled
    targets against the GPU direct sum."""
    _log("compare: Lagrange and Hermite treecodes on the Be-like mesh")
    t = tagi.Tree(x, y, z, leaf, box)
    res = {}
    for c in fields:
        k = c["kernel"]
        if k not in HERMITE_COMPARE:
            continue
        kap = c["kappa"] or 1.0
        ref = refs[k]
        res[k] = {}
        for target, forms in HERMITE_COMPARE[k].items():
            res[k][target] = {}
            for form, (th, deg) in forms.items():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t.upward(c["f"], w, deg, interpolation=form)
                torch.cuda.synchronize()
                up_ms = 1e3 * (time.perf_counter() - t0)
                u = t.convolve(k, kap, th, deg)
                ts = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    u = t.convolve(k, kap, th, deg)
                    torch.cuda.synchronize()
                    ts.append(1e3 * (time.perf_counter() - t0))
                ui = u[0, idx]
                st = t.stats()
                res[k][target][form] = {
                    "theta": th, "degree": deg, "convolve_ms": float(np.median(ts)),
                    "upward_ms": up_ms,
                    "rel_max": float((ui - ref).abs().max() / ref.abs().max()),
                    "rel_l2": float(torch.linalg.norm(ui - ref) / torch.linalg.norm(ref)),
                    "far_pairs": st["n_far_pairs"], "near_pairs": st["n_near_pairs"]}
            r = res[k][target]
            r["hermite_speedup"] = r["lagrange"]["convolve_ms"] / r["hermite"]["convolve_ms"]
    t.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="atom", choices=["atom", "cube"])
    ap.add_argument("--samples", type=int, default=2000, help="targets for the accuracy check")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the batched/mixed vs plain comparison on the benzene workload")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB five times (the "
                         "reference for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe_mib > 0:
        import torch
        n = args.copy_probe_mib * 2 ** 20 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 5}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures a single GPU; runs on more than one GPU are not part of this "
              "build (the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2003_01833_amd as tagi
    from workloads.configs import sample_targets

    torch.cuda.set_device(0)
    _log(f"bench: building workload {args.workload}")
    wl = make_workload(args.workload)
    n = wl["x"].size
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    x, y, z, w = dev(wl["x"]), dev(wl["y"]), dev(wl["z"]), dev(wl["w"])
    fields = [dict(c, f=dev(c["f"])) for c in wl["convs"]]
    outs = [torch.empty((1, n), dtype=torch.float64, device="cuda") for _ in fields]
    leaf = wl["leaf"]
    torch.cuda.synchronize()

    records = []

    def step():
        t = tagi.Tree(x, y, z, leaf, wl["box"])
        t.set_timing(True)
        stats = []
        for c, out in zip(fields, outs):
            t.upward(c["f"], w, c["degree"])
            t.convolve(c["kernel"], c["kappa"] or 1.0, c["theta"], c["degree"], alpha=1.0,
                       out=out)
            stats.append(t.stats())
        records.append((t.timing(), stats))
        t.close()

    for i in range(args.warmup):
        step()
        _log(f"bench: warmup step {i + 1}/{args.warmup} done")
    records.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for i in range(args.steps):
        ts = time.perf_counter()
        step()  # ends synchronised (phase timings are read, the tree is destroyed)
        step_ms.append(1e3 * (time.perf_counter() - ts))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _log(f"bench: {args.steps} timed steps in {elapsed:.3f} s")
    ms_per_step = 1e3 * elapsed / args.steps

    sts = records[-1][1]
    interactions = sum(st["far_interactions"] + st["near_interactions"] for st in sts)
    value = interactions / (ms_per_step / 1e3)
    # the N^2 pairs that the direct sums of one step would evaluate, per second
    direct_equivalent = n * n * len(fields) / (ms_per_step / 1e3)
    phases = {k: float(np.mean([r[0][k] for r in records])) for k in
              ("build_ms", "upward_ms", "lists_ms", "interact_ms", "combine_ms")}
    flops = sum(st["far_interactions"] * FLOPS[(c["kernel"], "far")] +
                st["near_interactions"] * FLOPS[(c["kernel"], "near")]
                for c, st in zip(fields, sts))
    gauss_near = gauss_far = 0
    for c in fields:
        if c["kernel"] == "coulomb_ss":
            sn, sf = coulomb_gauss_skipped(tagi, x, y, z, leaf, wl["box"], c["theta"], c["degree"])
            gauss_near += sn
            gauss_far += sf
    flops -= gauss_near * (FLOPS[("coulomb_ss", "near")] - COULOMB_NEAR_1R_FLOPS)
    flops -= gauss_far * (FLOPS[("coulomb_ss", "far")] - COULOMB_FAR_1R_FLOPS)
    interact_s = phases["interact_ms"] / 1e3
    achieved = flops / interact_s / 1e12
    launches = records[-1][0]["interact_launches"]

    # accuracy of the last step's outputs against the GPU direct sum at sampled targets
    idx = torch.from_numpy(sample_targets(n, min(args.samples, n), seed=4)).cuda()
    acc, refs = {}, {}
    for c, out in zip(fields, outs):
        f = c["f"]
        ref = tagi.direct(c["kernel"], x, y, z, f, w, x[idx].contiguous(), y[idx].contiguous(),
                          z[idx].contiguous(), f[idx].contiguous(), kappa=c["kappa"] or 1.0)
        refs[c["kernel"]] = ref
        u = out[0, idx]
        acc[c["kernel"]] = {"rel_l2": float(torch.linalg.norm(u - ref) / torch.linalg.norm(ref)),
                            "rel_max": float((u - ref).abs().max() / ref.abs().max())}

    stated = None
    if wl.get("stated"):
        th_s, deg_s, leaf_s = wl["stated"]
        t = tagi.Tree(x, y, z, leaf_s, wl["box"])
        stated = {"theta": th_s, "degree": deg_s, "leaf_size": leaf_s}
        for c in fields:
            t.upward(c["f"], w, deg_s)
            u = t.convolve(c["kernel"], c["kappa"] or 1.0, th_s, deg_s)[0, idx]
            ref = refs[c["kernel"]]
            stated[c["kernel"]] = {
                "rel_l2": float(torch.linalg.norm(u - ref) / torch.linalg.norm(ref)),
                "rel_max": float((u - ref).abs().max() / ref.abs().max())}
        t.close()

    comparison = hermite = None
    if not args.no_compare:
        if args.workload == "atom":
            hermite = compare_hermite(tagi, torch, x, y, z, w, fields, refs, idx, leaf, wl["box"])
        comparison = compare_batched(tagi, torch)

    cpu = None
    if not args.no_cpu_baseline:
        _log("bench: timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(wl, args.cpu_seconds)

    line = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "n_points": n, "leaf_size": leaf,
                   "settings": {c["kernel"]: {"theta": c["theta"], "degree": c["degree"],
                                              "far_pairs": st["n_far_pairs"],
                                              "near_pairs": st["n_near_pairs"]}
                                for c, st in zip(fields, sts)},
                   "n_leaves": sts[0]["n_leaves"], "interactions_per_step": interactions,
                   "coulomb_evaluations_without_gaussian": {"near": gauss_near,
                                                             "far": gauss_far}},
        "roofline": {"bound": "alu", "kernel": "k_interact", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "traffic_unit": "bytes per launch",
                     "launches_per_step": launches,
                     "avg_launch_ms": phases["interact_ms"] / max(launches, 1)},
        "cpu_baseline": cpu,
        "direct_equivalent_pairs_per_s": direct_equivalent,
        "phases_ms": phases,
        "ms_per_step_median": float(np.median(step_ms)),
        # a Green-iteration step on a fixed mesh reuses the tree and the lists:
        # upward passes, interaction kernels and combine only
        "ms_per_iteration_cached_tree": phases["upward_ms"] + phases["interact_ms"] + phases["combine_ms"],
        "accuracy_vs_direct": acc,
        "stated_setting_accuracy": stated,
        "batched_mixed_vs_plain": comparison,
        "hermite_vs_lagrange": hermite,
    }
    line["roofline"]["traffic"] = counter_traffic(line["config"])
    # the upward pass (proxy charges), against both the FP64 and the HBM roofline.
    # Per (source, approximable cluster) pair: barycentric basis values in three
    # dimensions, 4 flops per node (difference, divide, sum, normalise), the
    # (n+1)^2 products L_k1 L_k2, and one multiply-add per coefficient and charge
    # set; bytes: the source's coordinates and charges read once per cluster it
    # belongs to, and the proxy charges written once.
    up_flops = up_bytes = 0.0
    for c, st in zip(fields, sts):
        p1 = c["degree"] + 1
        sets = 2  # f w and w
        up_flops += st["upward_points"] * (12 * p1 + p1 * p1 + 2 * sets * p1 ** 3)
        up_bytes += st["upward_points"] * 8 * (3 + sets) + st["n_approx"] * 8 * sets * p1 ** 3
    up_s = phases["upward_ms"] / 1e3
    line["upward"] = {"ms_per_step": phases["upward_ms"],
                      "tflops": up_flops / up_s / 1e12,
                      "frac_fp64": up_flops / up_s / 1e12 / FP64_PEAK_TFLOPS,
                      "gbs": up_bytes / up_s / 1e9, "frac_hbm": up_bytes / up_s / 1e9 / 8000.0}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
