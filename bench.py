#!/usr/bin/env python3
"""Throughput of the coupled three-phase EHD lattice Boltzmann step on one GPU.

Workload: compound drop (core radius 60 inside shell radius 80) between
electrodes in a 1024 x 1024 box, electric capillary number 0.2, permittivity
ratios 2 and 0.5, conductivity ratios 3 and 0.3, charge relaxation time 0.6,
FP32 populations, a fixed number of potential sub-iterations per step.
One step = one coupled time step over every node (moments, stencils, charge,
all potential sub-iterations, chemical potential, fused collide-and-stream).

Prints ONE JSON line:  MLUPS (10^6 node updates per second), the dominant
kernel's HBM roofline figure measured live with HIP events, the FP64 variant,
the FP32-vs-FP64 field errors, and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def bytes_per_node(kernel, prec="fp32", Q=9, D=2):
    """Algorithmic HBM bytes per node and launch: what a kernel must read and
    write once (stencil neighbours and recomputed tile rings come from L2).
    T = macroscopic element size; populations f (3Q), g (Q), l (Q) are T
    wide, except FP16S: f^i_0 FP32 and the other populations 2 bytes.
    Q, D: the velocity set (9, 2 for D2Q9; 15, 3 for D3Q15)."""
    t = 8 if prec == "fp64" else 4
    s = {"fp64": 8, "fp32": 4, "fp16s": 2}[prec]                  # moving/flow/charge population size
    fpops = 3 * (t if prec != "fp16s" else 4) + 3 * (Q - 1) * s  # f: rest populations + moving ones
    pops = fpops + 2 * Q * s                                      # + g (Q) + l (Q)
    return {
        "moments": fpops + Q * s + 4 * t,                  # f, l in; phi, l-sum out
        "pre": (3 + 1 + D) * t + 3 * t,                    # phi, l-sum, E in; eps, q, R out
        "poisson": (Q + 1 + 1) * t + Q * t,                # h, eps, q in; h out (one sub-iteration)
        "poisson2": (Q + 1 + 1) * t + Q * t,               # the same for two or four sub-iterations per launch
        # a step's first four-sub-iteration launch with the charge step folded
        # in: h, phi, l-sum, E in; h, eps, q, R out (pre's traffic less the
        # eps and q it no longer re-reads)
        "poisson2_pre": (Q + 3 + 1 + D) * t + (Q + 3) * t,
        "mu": (Q + 1 + 1 + 3) * t + (1 + D + 3) * t,        # h, eps, psi, phi in; psi, E, mu out
        # pops in and out; phi and q of this and the previous step, mu, R, E,
        # the previous velocity in; the velocity out (p, rho on output steps only)
        "collide": 2 * pops + (3 + 3 + 3 + 1 + 1 + 1 + D + D) * t + D * t,
    }[kernel]


BYTES_PER_NODE_FP32 = {k: bytes_per_node(k) for k in ("moments", "pre", "poisson", "poisson2", "poisson2_pre", "mu",
                                                        "collide")}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in ("paper_2608_05787_amd/csrc/lbm_ehd_kernels.h", "paper_2608_05787_amd/csrc/lbm_ehd.hip"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, launch_nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, only
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_field_drop_1024.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or kernel not in t.get("kernels", {}):
        return None
    k = t["kernels"][kernel]
    return float(k["bytes_per_launch"]) if k.get("nodes") == launch_nodes else None


def copy_rate(mib=1024, reps=20):
    """Bytes moved per second (read + write) by a plain device-to-device copy
    of `mib` MiB, the streaming rate a memory-bound kernel can hope for."""
    import torch
    a = torch.ones(mib * 262144, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return round(2 * mib * 2 ** 20 / s / 1e9, 1)


def workload(n, sub, init_iters):
    """Fixed cold-start count, so that every precision starts from the same
    potential iterate."""
    from paper_2608_05787_amd import inputs
    p, init = inputs.field_compound_drop(n, sub=(sub, sub, 0.0), init_iters=init_iters, init_tol=0.0)
    return p, init


def run_gpu(p, init, precision, steps, warmup, profile_steps, tune_steps=0, config=-1):
    """Create, warm up, optionally autotune the launch configuration (bitwise
    the same results), then time `steps` steps with HIP events on the
    handle's stream.  Returns (sim, ms, per-kernel profile, diagnostics,
    tuning result or None)."""
    import torch
    from paper_2608_05787_amd import binding
    t0 = time.time()
    sim = binding.Sim(p, init, precision=precision)
    torch.cuda.synchronize()
    log("%s create (cold start) %.2fs" % (precision, time.time() - t0))
    tune = None
    if config >= 0:  # a fixed launch configuration (profiling the tuned one without the tuner's launches)
        sim.set_tuning(config)
        tune = {"config": config, "cached": False, "fixed": True}
    sim.step(warmup)
    torch.cuda.synchronize()
    if config < 0 and tune_steps > 0:
        tune = sim.autotune(steps=tune_steps)
        log("%s autotune: config %d, ms/step per config %s" % (precision, tune["config"],
                                                               ["%.4f" % v for v in tune["ms_per_step"]]))
    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    log("%s %d steps %.3f ms/step" % (precision, steps, ms / steps))
    prof = None
    if profile_steps > 0:
        sim.profile_begin()
        sim.step(profile_steps)
        prof = sim.profile_end()
    d = sim.diagnostics()
    return sim, ms, prof, d, tune


def cpu_baseline(p, init, budget_s):
    from oracle import Oracle
    q = dict(p, init_sub_max=0)  # bounded sample: no cold start
    t0 = time.time()
    o = Oracle(q, init)
    log("oracle create %.1fs" % (time.time() - t0))
    n_nodes = p["nx"] * p["ny"]
    steps, t0 = 0, time.time()
    while True:
        o.step(1)
        steps += 1
        el = time.time() - t0
        if el > budget_s or steps >= 200:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return {"value": n_nodes * steps / el / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "%dx%d field compound drop, %d FP64 oracle steps with %d potential "
                      "sub-iterations each (no cold start), %.1fs" % (p["nx"], p["ny"], steps, p["sub_max"], el)}


def field_errors(p, init, steps, precisions=("fp32", "fp16s")):
    """Error of each precision's fields against the FP64 instance of the same
    kernels (the FP64 instance matches the FP64 CPU oracle to ~1e-12), after
    the same fixed cold start and `steps` steps: relative L2 and element-wise
    (max |a - b| / max |b|) per field, the Sec. 4.4 deformation factors and
    the phase masses."""
    import torch
    from paper_2608_05787_amd import binding
    b = binding.Sim(p, init, precision="fp64")
    b.step(steps)
    fb = b.fields()
    db = b.diagnostics()
    del b
    res = {}
    for prec in precisions:
        a = binding.Sim(p, init, precision=prec)
        a.step(steps)
        fa = a.fields()
        out, mx = {}, {}
        for k in ("phi1", "phi2", "phi3", "ux", "uy", "p", "psi", "Ex", "Ey", "q", "mu1", "mu2", "mu3"):
            nb = float(torch.linalg.norm(fb[k]))
            out[k] = float(torch.linalg.norm(fa[k] - fb[k])) / nb if nb > 0 else 0.0
            mb = float(fb[k].abs().max())
            mx[k] = float((fa[k] - fb[k]).abs().max()) / mb if mb > 0 else 0.0
        out["max_norm"] = mx
        da = a.diagnostics()
        out["D_outer_abs"] = abs(da["D_outer"] - db["D_outer"])
        out["D_inner_abs"] = abs(da["D_inner"] - db["D_inner"])
        out["mass_rel"] = max(abs(da["mass%d" % i] - db["mass%d" % i]) / abs(db["mass%d" % i]) for i in (1, 2, 3))
        res[prec] = out
        del a
    res["D_outer_fp64"] = db["D_outer"]
    res["D_inner_fp64"] = db["D_inner"]
    return res


def batch_bench(n_inst, steps, sub, init_iters, graph_len=10, eager_steps=1000):
    """Parameter sweep (seeded sizes 128..512, field strengths, permittivity
    and conductivity ratios, half sheared): aggregate MLUPS of one batched
    handle replaying a captured graph of `graph_len` steps for `steps` steps,
    of one handle per instance stepped in turn for the same steps (sequential
    per-instance launches), of the grid-resident step (lbm_ehd_step_persistent)
    over the same batch and steps, and of the batched handle launched kernel
    by kernel (`eager_steps`), all FP32 on one side stream.  After the graph
    and sequential runs every instance of the batch must equal its separate
    run bitwise (all population families), and the persistent run the graph
    run."""
    import torch
    from paper_2608_05787_amd import binding, inputs
    cases = inputs.batch_sweep(n_inst=n_inst, sub=(sub, sub, 0.0), init_iters=init_iters)
    cfgs = [c[0] for c in cases]
    inits = [c[1] for c in cases]
    nodes = sum(c["nx"] * c["ny"] for c in cfgs)
    stream = torch.cuda.Stream()

    def timed(fn, reps):
        fn(graph_len)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(reps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    t0 = time.time()
    batch = binding.Sim(cfgs, inits, precision="fp32", stream=stream)
    torch.cuda.synchronize()
    log("batch create %.1fs, %d instances, %d nodes" % (time.time() - t0, n_inst, nodes))
    tune = batch.autotune(steps=10)
    log("batch autotune: config %d, ms/step per config %s" % (tune["config"],
                                                              ["%.3f" % v for v in tune["ms_per_step"]]))
    batch.graph(graph_len)
    ms_graph = timed(batch.step, steps)
    log("batch graph: %d steps %.1f ms" % (steps, ms_graph))
    sims = [binding.Sim(c, i, precision="fp32", stream=stream) for c, i in zip(cfgs, inits)]
    for sm in sims:
        sm.set_tuning(tune["config"])

    def seq(n):
        for _ in range(n):
            for sm in sims:
                sm.step(1)
    ms_seq = timed(seq, steps)
    log("sequential: %d steps %.1f ms" % (steps, ms_seq))
    equal = all(torch.equal(batch.populations(fam, inst=i), sm.populations(fam))
                for i, sm in enumerate(sims) for fam in "fglh")
    d_batch = [batch.diagnostics(i) for i in range(n_inst)]
    del sims
    torch.cuda.empty_cache()
    # the grid-resident step (cooperative launches of up to 256 steps each)
    # over the same batch and steps, against the graph-replayed handle
    pers = binding.Sim(cfgs, inits, precision="fp32", stream=stream)
    pers.set_tuning(tune["config"])
    ms_pers = timed(pers.step_persistent, steps)
    log("persistent: %d steps %.1f ms" % (steps, ms_pers))
    pers_equal = all(torch.equal(batch.populations(fam, inst=i), pers.populations(fam, inst=i))
                     for i in range(n_inst) for fam in "fglh")
    # where its step goes: 100 more steps with the stage clocks on
    pers.set_persistent_timing(True)
    pers.step_persistent(100)
    pers_stage_us = {k: round(v, 1) for k, v in pers.persistent_stage_times().items()}
    log("persistent stage us per step %s" % pers_stage_us)
    del pers
    torch.cuda.empty_cache()
    batch.graph(0)
    ms_eager = timed(batch.step, eager_steps)
    del batch
    mlups = lambda ms, n: round(nodes * n / (ms * 1e-3) / 1e6, 1)
    return {"instances": n_inst, "nodes": nodes, "steps": steps, "potential_subiterations": sub,
            "graph_steps": graph_len, "mlups_graph": mlups(ms_graph, steps),
            "mlups_batched_eager": mlups(ms_eager, eager_steps), "eager_steps": eager_steps,
            "mlups_sequential": mlups(ms_seq, steps), "speedup_graph_vs_sequential": round(ms_seq / ms_graph, 2),
            "mlups_persistent": mlups(ms_pers, steps), "persistent_equals_graph_bitwise": pers_equal,
            "persistent_stage_us": pers_stage_us,
            "instances_equal_separate_runs_bitwise": equal,
            "max_sum_dev_worst": max(d["max_sum_dev"] for d in d_batch),
            "nonfinite_total": sum(d["nonfinite"] for d in d_batch),
            "tuning": tune}


def adaptive_bench(p, init, steps, warmup, tol, kmax=64):
    """The headline workload with residual-controlled potential
    sub-iterations (stop once the relative change of the potential over an
    iteration is below tol): mean sub-iterations per step and MLUPS at that
    count (one launch and one control pass per sub-iteration)."""
    import torch
    from paper_2608_05787_amd import binding
    q = dict(p, sub_min=1, sub_max=kmax, sub_tol=tol)
    sim = binding.Sim(q, init, precision="fp32")
    sim.step(warmup)
    k0 = sim.scalars()["k_total"]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    k1 = sim.scalars()["k_total"]
    d = sim.diagnostics()
    # the fixed-count run over the same steps: deformation and fields
    fix = binding.Sim(p, init, precision="fp32")
    fix.step(warmup + steps)
    df = fix.diagnostics()
    fa, fb = sim.fields(), fix.fields()
    diff = {k: float((fa[k] - fb[k]).abs().max() / fb[k].abs().max()) for k in ("phi1", "ux", "psi", "Ey", "q", "mu1")}
    nodes = p["nx"] * p["ny"]
    return {"sub_tol": tol, "sub_max": kmax, "steps": steps, "mean_k": (k1 - k0) / steps,
            "mlups": round(nodes * steps / (ms * 1e-3) / 1e6, 1), "ms_per_step": ms / steps,
            "last_residual": d["residual"], "status": d["status"],
            "fixed_k": p["sub_max"], "fixed_k_last_residual": df["residual"],
            "D_outer_diff_vs_fixed_k": abs(d["D_outer"] - df["D_outer"]),
            "D_inner_diff_vs_fixed_k": abs(d["D_inner"] - df["D_inner"]),
            "field_max_norm_diff_vs_fixed_k": diff}


def d3q15_bench(n, steps, warmup, sub, init_iters, profile_steps):
    """The field-driven compound drop on the D3Q15 lattice (n^3 box, radii
    0.3125 n and 0.234 n): FP32 MLUPS, per-kernel average launch times and
    their algorithmic GB/s, and the FP16S and FP64 rates."""
    import torch
    from paper_2608_05787_amd import inputs
    p, init = inputs.field_compound_drop3d(n, r_shell=0.3125 * n, r_core=0.234375 * n, sub=(sub, sub, 0.0),
                                           init_iters=init_iters)
    nodes = n ** 3
    out = {"workload": "field compound drop %d^3 on D3Q15 (electrodes, Ca_e 0.2, eps ratios 2/0.5, "
                       "sigma ratios 3/0.3, radii %.0f/%.0f)" % (n, 0.3125 * n, 0.234375 * n),
           "nodes": nodes, "potential_subiterations": sub}
    for prec in ("fp32", "fp16s", "fp64"):
        k = steps if prec != "fp64" else max(steps // 2, 1)
        sim, ms, prof, diag, _ = run_gpu(p, init, prec, k, warmup, profile_steps if prec == "fp32" else 0)
        step_bytes = sum(bytes_per_node(kk, prec, 15, 3) * (sub if kk == "poisson" else 1)
                         for kk in ("moments", "pre", "poisson", "mu", "collide"))
        out[prec] = {"mlups": round(nodes * k / (ms * 1e-3) / 1e6, 1), "ms_per_step": ms / k,
                     "bytes_per_node_update": step_bytes,
                     "effective_gbs": round(step_bytes * nodes * k / (ms * 1e-3) / 1e9, 1)}
        if prof:
            kern = {}
            for name, (tot, cnt) in prof.items():
                if cnt:
                    avg = 1e3 * tot / cnt
                    kern[name] = {"avg_us": round(avg, 2), "launches": cnt}
                    if name in ("moments", "pre", "poisson", "mu", "collide"):
                        kern[name]["gbs"] = round(bytes_per_node(name, prec, 15, 3) * nodes / (avg * 1e-6) / 1e9, 1)
            out[prec]["kernels"] = kern
            out[prec]["diagnostics"] = {kk: diag[kk] for kk in ("max_sum_dev", "D_outer", "D_inner", "nonfinite")}
        del sim
        torch.cuda.empty_cache()
    return out


def gradient_bench(n, steps, sub, init_iters, every):
    """Gradient of the outer deformation after `steps` steps with respect to
    the five parameters on the adjoint workload (n x n, radii 40/30) by the
    reverse sweep: lbm_ehd_record (the FP32 forward with a checkpoint every
    `every` steps) then lbm_ehd_adjoint (segments recomputed from their
    checkpoints, step adjoints backwards, then create's).  Times are against
    the plain FP32 forward run of the same length from create, in the launch
    configuration the autotuner picks for it (the recording forward uses the
    same); the FP32 gradient is compared with the FP64 sweep's."""
    import torch
    from paper_2608_05787_amd import autograd, binding, inputs
    p, init = inputs.field_compound_drop(n, r_shell=40.0, r_core=30.0, sub=(sub, sub, 0.0),
                                         init_iters=init_iters, init_tol=0.0)
    warm = binding.Sim(p, init, precision="fp32")  # first-use costs stay out of the timings
    warm.step(10)
    cfg = warm.autotune(steps=10)["config"]  # the forward runs in its fastest launch configuration
    torch.cuda.synchronize()
    del warm
    t0 = time.time()
    fwd = binding.Sim(p, init, precision="fp32")
    fwd.set_tuning(cfg)
    fwd.step(steps)
    phi = fwd.fields(["phi1"])["phi1"]
    torch.cuda.synchronize()
    t_fwd = time.time() - t0
    del fwd
    w = (1.0 - phi.double()).clone().requires_grad_(True)
    D = autograd.deformation(autograd.drop_indicator(w))
    D.backward()
    seed = {"phi1": -w.grad.detach()}
    torch.cuda.synchronize()
    t0 = time.time()
    rec = binding.Sim(p, init, precision="fp32")
    rec.set_tuning(cfg)
    rec.record(steps, every)
    torch.cuda.synchronize()
    t_rec = time.time() - t0
    t0 = time.time()
    g = rec.adjoint(steps, seed, every)
    torch.cuda.synchronize()
    t_adj = time.time() - t0
    del rec
    torch.cuda.empty_cache()
    ref = binding.Sim(p, init, precision="fp64")
    torch.cuda.synchronize()
    t0 = time.time()
    g64 = ref.adjoint(steps, seed, every)
    torch.cuda.synchronize()
    t_adj64 = time.time() - t0
    del ref
    torch.cuda.empty_cache()
    # the FP64 forward's own deformation: how far the FP32 forward already is
    f64 = binding.Sim(p, init, precision="fp64")
    f64.step(steps)
    w64 = 1.0 - f64.fields(["phi1"], dtype=torch.float64)["phi1"]
    D64 = float(autograd.deformation(autograd.drop_indicator(w64)))
    del f64
    torch.cuda.empty_cache()
    rel = [abs(a - b) / abs(b) if b != 0 else abs(a) for a, b in zip(g, g64)]
    gmax = max(abs(b) for b in g64)
    return {"workload": "field compound drop %dx%d, radii 40/30, %d steps, %d potential sub-iterations, "
                        "cold start %d iterations" % (n, n, steps, sub, init_iters),
            "method": "reverse sweep, FP32, checkpoint every %d steps" % every,
            "forward_launch_config": cfg,
            "D_outer": float(D.detach()), "dD_dtheta": g, "dD_dtheta_fp64_sweep": g64,
            "rel_diff_fp32_vs_fp64": rel,
            "diff_fp32_vs_fp64_over_max_component": [abs(a - b) / gmax for a, b in zip(g, g64)],
            "D_outer_fp64_forward": D64, "rel_diff_D_fp32_vs_fp64_forward": abs(float(D.detach()) - D64) / abs(D64) if D64 else None,
            "adjoint_fp64_s": round(t_adj64, 4),
            "forward_s": round(t_fwd, 4), "record_s": round(t_rec, 4), "adjoint_s": round(t_adj, 4),
            "adjoint_over_forward": round(t_adj / t_fwd, 2),
            "record_plus_adjoint_over_forward": round((t_rec + t_adj) / t_fwd, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--sub", type=int, default=4, help="potential sub-iterations per step")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--tune-steps", type=int, default=20,
                    help="steps timed per launch configuration by the autotuner (0: default configuration)")
    ap.add_argument("--config", type=int, default=-1,
                    help="launch configuration of the 1024^2 legs, in place of the autotuner (-1: tune)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--error-steps", type=int, default=500)
    ap.add_argument("--init-iters", type=int, default=4000, help="cold-start potential iterations")
    ap.add_argument("--batch-instances", type=int, default=64, help="0 skips the parameter-sweep leg")
    ap.add_argument("--batch-steps", type=int, default=10000)
    ap.add_argument("--adaptive-tol", type=float, default=1e-7,
                    help="residual tolerance of the residual-controlled leg (0 skips it)")
    ap.add_argument("--grad-steps", type=int, default=5000, help="0 skips the gradient leg")
    ap.add_argument("--grad-every", type=int, default=250, help="checkpoint interval of the reverse sweep")
    ap.add_argument("--n3", type=int, default=128, help="edge of the D3Q15 box (0 skips the 3-D leg)")
    ap.add_argument("--d3q15-only", action="store_true",
                    help="run only the D3Q15 leg (for profiling) and print its JSON object")
    ap.add_argument("--gradient-only", action="store_true",
                    help="run only the gradient leg (for profiling) and print its JSON object")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the parameter-sweep leg and print its JSON object")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only (there is no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2608_05787_amd import binding
    binding.load()

    if args.d3q15_only:
        print(json.dumps({"d3q15": d3q15_bench(args.n3, max(args.steps // 4, 10), max(args.warmup // 4, 5), args.sub,
                                               1000, args.profile_steps)}), flush=True)
        return

    if args.gradient_only:
        print(json.dumps({"gradient": gradient_bench(512, args.grad_steps, args.sub, 2000, args.grad_every)}),
              flush=True)
        return

    if args.batch_only:
        print(json.dumps({"batch_sweep": batch_bench(args.batch_instances, args.batch_steps, args.sub, 1000)}),
              flush=True)
        return

    if args.calib_copy_mib > 0:
        a = torch.ones(args.calib_copy_mib * 262144, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calib_copy_mib)
        del a, b
    copy_gbs = copy_rate() if args.profile_steps > 0 else None
    p, init = workload(args.n, args.sub, args.init_iters)
    nodes = p["nx"] * p["ny"]
    sim, ms, prof, diag, tune = run_gpu(p, init, "fp32", args.steps, args.warmup, args.profile_steps,
                                        args.tune_steps, args.config)
    mlups = nodes * args.steps / (ms * 1e-3) / 1e6
    k_mean = args.sub

    roofline = None
    kernels = {}
    if prof:
        for k, (tot, cnt) in prof.items():
            if cnt:
                kernels[k] = {"avg_us": 1e3 * tot / cnt, "launches": cnt, "share": 0.0}
        total = sum(v["avg_us"] * v["launches"] for v in kernels.values())
        for v in kernels.values():
            v["share"] = v["avg_us"] * v["launches"] / total
        dom = max((k for k in kernels if k in BYTES_PER_NODE_FP32),
                  key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
        bpl = BYTES_PER_NODE_FP32[dom] * nodes
        avg_s = kernels[dom]["avg_us"] * 1e-6
        achieved = bpl / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "bytes_per_launch": bpl, "bytes_per_node": BYTES_PER_NODE_FP32[dom],
                    "traffic": measured_traffic(dom, nodes),
                    # context: a plain device copy (read + write) on the same GPU
                    "copy_gbs": copy_gbs,
                    "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None}
        for k, v in kernels.items():
            if k in BYTES_PER_NODE_FP32:
                v["gbs"] = round(BYTES_PER_NODE_FP32[k] * nodes / (v["avg_us"] * 1e-6) / 1e9, 1)
    # potential launches of a step: one single launch when K is odd, then
    # LDS-tiled launches of four sub-iterations (tall tiles, 4-byte
    # arithmetic) and of two; K singles when the tuner chose single launches
    def launches(cfg):
        """(launches of the LDS-tiled potential kernel, single launches) per
        step: one single launch when K is odd, then four sub-iterations per
        launch on tall tiles while four remain, then two; K singles when the
        configuration asks for single launches."""
        if cfg & 2:
            return 0, args.sub
        n1, rest = args.sub % 2, args.sub - args.sub % 2
        quads = rest // 4 if cfg & 8 else 0
        return quads + (rest - 4 * quads) // 2, n1

    def step_bytes(prec, cfg):
        """Algorithmic bytes per node of one step in configuration cfg: with
        tall tiles and an even K >= 4 the charge step rides on the first
        four-sub-iteration launch."""
        n2, n1 = launches(cfg)
        fold = bool(cfg & 8) and not cfg & 2 and args.sub >= 4 and args.sub % 2 == 0
        count = {"moments": 1, "pre": 0 if fold else 1, "poisson": n1, "poisson2": n2 - fold,
                 "poisson2_pre": int(fold), "mu": 1, "collide": 1}
        return sum(bytes_per_node(k, prec) * c for k, c in count.items())

    cfg32 = tune["config"] if tune else 0
    variants = {"fp32": {"mlups": round(mlups, 1), "ms_per_step": ms / args.steps, "launch_config": cfg32,
                         "bytes_per_node_update": step_bytes("fp32", cfg32)}}
    errors = None
    if not args.no_variants:
        del sim
        _, ms64, _, _, t64 = run_gpu(p, init, "fp64", max(args.steps // 2, 1), args.warmup // 2, 0, args.tune_steps,
                                     args.config)
        cfg64 = t64["config"] if t64 else 0
        variants["fp64"] = {"mlups": round(nodes * max(args.steps // 2, 1) / (ms64 * 1e-3) / 1e6, 1),
                            "ms_per_step": ms64 / max(args.steps // 2, 1), "launch_config": cfg64,
                            "bytes_per_node_update": step_bytes("fp64", cfg64)}
        _, ms16, _, _, t16 = run_gpu(p, init, "fp16s", args.steps, args.warmup, 0, args.tune_steps, args.config)
        cfg16 = t16["config"] if t16 else 0
        variants["fp16s"] = {"mlups": round(nodes * args.steps / (ms16 * 1e-3) / 1e6, 1),
                             "ms_per_step": ms16 / args.steps, "launch_config": cfg16,
                             "bytes_per_node_update": step_bytes("fp16s", cfg16)}
        log("field errors FP32 / FP16S vs FP64 after %d steps" % args.error_steps)
        errors = field_errors(p, init, args.error_steps)

    adaptive = None
    if args.adaptive_tol > 0 and not args.no_variants:
        log("residual-controlled potential sub-iterations, tol %g" % args.adaptive_tol)
        adaptive = adaptive_bench(p, init, max(args.steps // 4, 10), args.warmup, args.adaptive_tol)
        log("mean K %.2f at %.1f MLUPS" % (adaptive["mean_k"], adaptive["mlups"]))

    batch = None
    if args.batch_instances > 0 and not args.no_variants:
        log("batched parameter sweep")
        batch = batch_bench(args.batch_instances, args.batch_steps, args.sub, 1000)

    grad = None
    if args.grad_steps > 0 and not args.no_variants:
        log("gradient (adjoint workload)")
        grad = gradient_bench(512, args.grad_steps, args.sub, 2000, args.grad_every)

    d3 = None
    if args.n3 > 0 and not args.no_variants:
        log("D3Q15 leg")
        d3 = d3q15_bench(args.n3, max(args.steps // 4, 10), max(args.warmup // 4, 5), args.sub, 1000,
                         args.profile_steps)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(p, init, args.cpu_seconds)

    out = {
        "metric": "coupled MLUPS (FP32 populations, fixed potential sub-iterations)",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "field compound drop %dx%d (electrodes, Ca_e 0.2, eps ratios 2/0.5, "
                               "sigma ratios 3/0.3, radii 80/60)" % (args.n, args.n),
                   "nodes": nodes, "potential_subiterations": k_mean, "precision": "fp32",
                   "algorithmic_bytes_per_node_update": step_bytes("fp32", cfg32),
                   "mean_k_residual_controlled": adaptive["mean_k"] if adaptive else None},
        "tuning": tune,
        "roofline": roofline,
        "kernels": kernels,
        "variants": variants,
        "errors_vs_fp64": errors,
        "residual_controlled": adaptive,
        "batch_sweep": batch,
        "gradient": grad,
        "d3q15": d3,
        "diagnostics": {k: diag[k] for k in ("max_sum_dev", "residual", "D_outer", "D_inner", "nonfinite")},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
