#!/usr/bin/env python3
"""Throughput of the D2Q9 KBC stream-and-collide step on one MI355X.

Workload (the roofline run): one periodic 16384 x 16384 lattice, a seeded
divergence-free random initial field with E(k) ~ k^4 exp(-2 (k/32)^2),
u_rms = 0.05, rho = 1, nu = 1e-4, Grad initialisation with central
differences; KBC model B, populations stored as FP32 deviations, FP32
arithmetic.  The library's default launch runs two fused pull-stream +
collide steps per kernel launch (the first step's result stays in LDS), so
the state crosses HBM once per two steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

prints one JSON line.  `value` is lattice updates per second (MLUPS) over the
K timed steps.  `roofline` describes the dominant kernel: with two fused
steps per launch it is bound by vector-ALU issue, so `bound` is "alu" and
`achieved` counts the FP32 operations of its compiled collision against the
published FP32 vector peak; the same object gives the HBM side per launch
(72 B per node per launch over the launch time, against 8 TB/s).  With
--fusion 1 (one step per launch) the kernel is HBM-bound and `bound` is
"hbm".  `cpu_baseline` times the FP64 CPU oracle on a bounded sample of the
same workload on all host cores (up to 16) and on one core.
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS and % of HBM roofline (KBC fwd, adjoint) at stated error vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"f16": 36, "f32": 72, "f64": 144}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_traffic.json")
_CSRC = os.path.join(ROOT, "paper_1507_02509_amd", "csrc")
STEP_SOURCES = [os.path.join(_CSRC, f)
                for f in ("kbc_step.hip", "kbc_step2.hip", "kbc_tile.hpp", "kbc_tile2.hpp", "kbc_device.hpp")]
# Floating-point operations of one KBC-B collision per node as compiled for
# gfx950 (adds, multiplies, reciprocals and conversions count one, FMAs two),
# counted in the single-step kernel's code: "compiled-instruction FLOPs", not
# a minimal operation count of the method.  The vector peaks are MI355X's
# published ones; the FP32 one assumes packed FP32 (two lanes per
# instruction), which this library never issues, so at most half of it is
# attainable here.
FLOPS_PER_NODE_STEP = {"f32": 266, "f16": 302, "f64": 382}
VECTOR_PEAK_TFLOPS = {"f32": 157.3, "f16": 157.3, "f64": 78.6}
VALU_ISSUE_PEAK = 256 * 64 * 2.4e9   # lane-instructions/s: 256 CUs, 64 lanes, nominal clock
# untimed steps before each extra measurement, so that none is timed while the
# clock is still ramping up after the previous one's host-side work
EXTRA_WARMUP = 20
ADJOINT_SOURCES = [os.path.join(_CSRC, f)
                   for f in ("kbc_adjoint.hip", "kbc_adjoint.hpp", "kbc_tile.hpp", "kbc_device.hpp")]


def kernel_digest(sources=STEP_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str, section: str = "step", field: str = "bytes_per_launch"):
    """A per-launch figure (HBM bytes by default) from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = rec.get(section, {})
    sources = STEP_SOURCES if section == "step" else ADJOINT_SOURCES
    if rec.get("kernel_digest") != kernel_digest(sources):
        return None
    entry = rec.get("workloads", {}).get(key)
    return None if entry is None else entry.get(field)


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(sim, steps: int, warmup: int):
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    sim.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    return t0.elapsed_time(t1) / steps, wall


def make_sim(n, form, collision, variant, nu, seed, k0, device):
    from paper_1507_02509_amd import inputs
    from paper_1507_02509_amd.sim import Sim, beta_from_nu
    ux, uy = inputs.spectral(n, k0, 0.05, seed=seed, device=device)
    sim = Sim(n, n, beta_from_nu(nu), collision=collision, variant=variant, form=form, device=device)
    sim.init(ux, uy)
    del ux, uy
    return sim


def time_adjoint(n, nu, seed, k0, dev, steps=20):
    """The adjoint step kernel on the same lattice (state f^n fixed, random
    adjoint field): 9 state loads + 9 adjoint loads + 9 adjoint stores."""
    import torch
    sim = make_sim(n, "f32", "kbc", "B", nu, seed, k0, dev)
    la, lb = sim.new_adjoint(), sim.new_adjoint()
    la.normal_()
    acc = torch.zeros(1, dtype=torch.float64, device=dev)
    state = sim.state_buffer()
    for _ in range(EXTRA_WARMUP):
        sim.adjoint_step(state, la, lb, acc)
        la, lb = lb, la
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        sim.adjoint_step(state, la, lb, acc)
        la, lb = lb, la
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del sim, la, lb
    torch.cuda.empty_cache()
    return ms


C5 = {"n": 512, "steps": 2000, "variant": "D", "gamma_guard": 1e-4, "nu": 1e-3, "form": "f32"}


def time_c5(dev):
    """Forward and backward of the differentiable rollout on the adjoint
    workload: 512^2 decaying turbulence (k0 = 8, u_rms = 0.05, nu = 1e-3),
    FP32, 2000 steps, sqrt(N) checkpoints, loss 1/2 |u(T) - u_t|^2.  The
    collision is KBC-D with stabiliser guard 1e-4: the KBC configuration whose
    2000-step gradient is verified (central finite differences of the FP64
    forward and the FP32 vs FP64 gradient, and the FP64 discrete adjoint
    against the oracle's over 50 steps); with KBC-B and the default guard the
    exact gradient grows to ~1e30 over 2000 steps and carries no meaning.
    The gradient is checked to be finite and its norm reported."""
    import torch
    from paper_1507_02509_amd import inputs
    from paper_1507_02509_amd.autograd import rollout
    from paper_1507_02509_amd.sim import beta_from_nu
    n, nsteps = C5["n"], C5["steps"]
    ux0, uy0 = (torch.from_numpy(a).to(dev) for a in inputs.spectral(n, 8, 0.05, seed=5))
    tx, ty = (torch.from_numpy(a).to(dev) for a in inputs.spectral(n, 8, 0.03, seed=55))
    out = {}
    for rep in range(2):
        u0x = ux0.clone().requires_grad_(True)
        u0y = uy0.clone().requires_grad_(True)
        b = torch.tensor(beta_from_nu(C5["nu"]), dtype=torch.float64, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ux, uy = rollout(u0x, u0y, b, nsteps, form=C5["form"], variant=C5["variant"],
                            gamma_guard=C5["gamma_guard"])
        loss = 0.5 * (((ux - tx) ** 2).sum() + ((uy - ty) ** 2).sum())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gnorm = float(torch.sqrt((u0x.grad ** 2).sum() + (u0y.grad ** 2).sum()))
        if not (np.isfinite(gnorm) and np.isfinite(b.grad.item())):
            raise RuntimeError(f"non-finite rollout gradient (|grad u0| {gnorm}, dL/dbeta {b.grad.item()})")
        out = {"config": f"KBC-{C5['variant']}, guard {C5['gamma_guard']:g}, {C5['form']}, {n}^2, {nsteps} steps",
               "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
               "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
               "grad_u0_norm": gnorm, "dL_dbeta": b.grad.item(), "loss": loss.item()}
    return out


def time_slab(dev, steps=200, slabs=8):
    """One GPU's share of the 16384^2 workload split in y over `slabs` GPUs:
    a 16384 x (16384 / slabs) slab whose rows -2, -1 and ny, ny + 1 come
    from halo buffers (lbm_set_halo).  Before every launch of two fused steps
    the halo is refreshed the way a multi-GPU run would do it, here from the
    slab's own edge rows (lbm_get_edge_rows, then two device copies standing
    in for the sends), all inside the timed region; against the same slab as
    a periodic lattice with no exchange."""
    import torch
    n = 16384
    h = n // slabs
    sim = make_sim(n, "f32", "kbc", "B", 1e-4, 3, 32, dev)
    state = sim.state_buffer()[:h].clone()
    del sim
    torch.cuda.empty_cache()
    from paper_1507_02509_amd.sim import Sim, beta_from_nu
    res = {"slab": f"{n} x {h}", "slabs": slabs}
    for mode in ("periodic", "halo"):
        s = Sim(n, h, beta_from_nu(1e-4), collision="kbc", variant="B", form="f32", device=dev)
        s.init(np.zeros((h, n)), np.zeros((h, n)), mode="eq")
        s.state_buffer().copy_(state)
        lo, hi = s.halo_buffers()
        send_lo, send_hi = s.halo_buffers()

        def launch():
            if mode == "halo":
                s.edge_rows(send_lo, send_hi)
                lo.copy_(send_hi)
                hi.copy_(send_lo)
            s.step(2)
        if mode == "halo":
            s.set_halo(lo, hi)
        # 100 warm-up steps: after 10 this slab measured 117.6 G node-steps/s,
        # after 200 (in another run) 141.6, the clock's ramp after the
        # previous benchmark's host-side work
        for _ in range(50):
            launch()
        torch.cuda.synchronize()
        launches = max(steps, 200) // 2
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            launch()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (2 * launches)
        res[mode] = {"ms_per_step": round(ms, 4), "mlups": round(n * h / (ms * 1e-3) / 1e6, 1)}
        del s
        torch.cuda.empty_cache()
    # bytes that would cross to the two neighbours per launch of two steps
    res["exchange_bytes_per_launch"] = 2 * 2 * 9 * n * 4
    res["halo_over_periodic_time"] = round(res["halo"]["ms_per_step"] / res["periodic"]["ms_per_step"], 3)
    return res


def time_ensemble(dev, steps=60, persistent_steps=2000):
    """The uneven ensemble: 256 members, N in {128, 256, 512, 1024}, KBC-B FP32.
    (a) the library's default launch (one batched launch over all members'
    tiles per two fused steps), `steps` steps; (b) the workload as stated:
    `persistent_steps` steps in ONE persistent launch (grid barrier between
    pairs of steps) with the launch configuration the autotuner picks for the
    persistent mode on this ensemble (timed on the ensemble itself, state
    restored), checked for barrier give-ups afterwards."""
    import torch
    from paper_1507_02509_amd import autotune, inputs
    from paper_1507_02509_amd.ensemble import Ensemble, make_members
    specs = inputs.ensemble_members(256, master_seed=4)
    sims = make_members(specs, form="f32", device=dev)
    ens = Ensemble(sims)
    nodes = ens.nodes
    ens.step(10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ens.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    spl = ens.fusion
    res = {"members": 256, "nodes": nodes, "ms_per_step": round(ms, 4),
           "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "steps_per_launch": spl,
           "hbm_frac": round(72 * nodes / (spl * ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "launch": "one batched launch over all members per " + ("two steps" if spl == 2 else "step")}
    best, _ = autotune.tune_ensemble(ens, steps=10, reps=2, persistent=True, use_cache=False)
    blocks = ens.blocks
    ens.step(2, persistent=True)
    torch.cuda.synchronize()
    e0.record()
    ens.step(persistent_steps, persistent=True)
    e1.record()
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1) / persistent_steps
    ens.check()
    d = sims[255].diagnostics()
    res["persistent"] = {"steps": persistent_steps, "launches": 1, "grid_workgroups": blocks,
                         "autotuned_config": list(best), "ms_per_step": round(pms, 4),
                         "mlups": round(nodes / (pms * 1e-3) / 1e6, 1),
                         "member_255_nonfinite": d["n_nonfinite"]}
    ens.free()
    del ens, sims
    torch.cuda.empty_cache()
    return res


def form_errors(n, nu, seed, k0, dev, steps=10):
    """Velocity error of the FP32 and FP16 deviation forms against the FP64
    form after `steps` steps of the same workload (max |du| / max |u|)."""
    import torch
    res = {}
    ref = make_sim(n, "f64", "kbc", "B", nu, seed, k0, dev).step(steps)
    _, rx, ry = ref.moments()
    del ref
    for form in ("f32", "f16"):
        s = make_sim(n, form, "kbc", "B", nu, seed, k0, dev).step(steps)
        _, ux, uy = s.moments()
        del s
        e = max(float((ux - rx).abs().max() / rx.abs().max()), float((uy - ry).abs().max() / ry.abs().max()))
        res[form] = e
        del ux, uy
        torch.cuda.empty_cache()
    return {"steps": steps, "u_rel_err_vs_f64": res}


def _oracle_mlups(p, f, target_s: float):
    """Node updates per second of the oracle's step on state f, over about
    target_s seconds (at least two steps)."""
    import oracle
    t0 = time.perf_counter()
    f1 = oracle.step(p, f)
    one = time.perf_counter() - t0
    nsteps = max(1, int(target_s / max(one, 1e-3)) - 1)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        f1 = oracle.step(p, f1)
    dt = time.perf_counter() - t0 + one
    return p.nx * p.ny * (nsteps + 1) / dt / 1e6, nsteps + 1, dt


def cpu_baseline(n: int, nu: float, seed: int, k0: float):
    """The FP64 oracle (unmodified) on slabs of the same workload, treated as
    periodic lattices of the same row length (the same per-node work): KBC-B
    on all host cores (up to 16) over a 2048-row slab for about 12 s, on one
    core over a 128-row slab for about 5 s, and LBGK likewise (about 4 s and
    3 s) for the oracle's KBC / LBGK time ratio."""
    import oracle
    from paper_1507_02509_amd import inputs
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = max(1, min(threads, 16))
    ux, uy = inputs.spectral(n, k0, 0.05, seed=seed, device="cuda")
    beta = 1.0 / (6.0 * nu + 1.0)
    res = {}
    for rows, nt, label, tk, tl in ((2048, threads, "all", 12.0, 4.0), (128, 1, "one", 5.0, 3.0)):
        vx = np.ascontiguousarray(ux[:rows].cpu().numpy())
        vy = np.ascontiguousarray(uy[:rows].cpu().numpy())
        pk = oracle.Params(n, rows, beta, collision=oracle.KBC, variant=oracle.KBC_B, threads=nt)
        pl = oracle.Params(n, rows, beta, collision=oracle.LBGK, threads=nt)
        f = oracle.init(pk, vx, vy)
        res[label] = (rows, nt, _oracle_mlups(pk, f, tk), _oracle_mlups(pl, f, tl))
    rows, nt, (k_all, steps_all, dt_all), (l_all, _, _) = res["all"]
    rows1, _, (k_one, steps_one, dt_one), (l_one, _, _) = res["one"]
    return {"value": round(k_all, 3), "unit": "MLUPS", "cores": nt, "kind": "oracle",
            "sample": f"KBC-B FP64 oracle, {steps_all} steps of a periodic {n} x {rows} slab of the "
                      f"same seeded field ({n * rows * steps_all / 1e6:.0f} M node updates, {dt_all:.1f} s); "
                      f"one core: {steps_one} steps of a {n} x {rows1} slab ({dt_one:.1f} s); LBGK on the same "
                      f"slabs for the ratio",
            "one_core": {"value": round(k_one, 3), "unit": "MLUPS", "cores": 1},
            "lbgk": {"value": round(l_all, 3), "one_core_value": round(l_one, 3), "unit": "MLUPS"},
            "kbc_over_lbgk_time": {"all_cores": round(l_all / k_all, 3), "one_core": round(l_one / k_one, 3)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--form", default="f32", choices=["f16", "f32", "f64"])
    ap.add_argument("--variant", default="B")
    ap.add_argument("--fusion", type=lambda v: tuple(int(x) for x in v.split(",")), default=None,
                    help="steps per launch [,fused tile rows], e.g. 1 or 2,16 (default: the library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="forms,lbgk,exact,copy,adjoint,rollout,ensemble,slab,accuracy",
                    help="comma-separated extra measurements")
    ap.add_argument("--extra-steps", type=int, default=50,
                    help="timed steps for the other forms and the LBGK baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    dev = "cuda:0"
    n, nu, seed, k0 = args.n, 1e-4, 3, 32
    workload = f"d2q9_kbc{args.variant}_turbulence_{n}x{n}_k0_{k0}_nu_1e-4"

    progress(f"init {n}x{n} {args.form} KBC-{args.variant}")
    sim = make_sim(n, args.form, "kbc", args.variant, nu, seed, k0, dev)
    if args.fusion is not None:
        sim.set_fusion(*args.fusion)
    spl = sim.fusion
    rows = sim.fusion_rows
    d0 = sim.diagnostics()
    ms, wall = time_steps(sim, args.steps, args.warmup)
    progress(f"timed {args.steps} steps: {ms:.4f} ms/step")
    d_main = sim.diagnostics()      # the headline run's end state (the extras reuse d)
    del sim
    torch.cuda.empty_cache()
    nodes = n * n
    mlups = nodes / (ms * 1e-3) / 1e6
    launch_ms = ms * spl      # one launch advances spl steps (an odd step count adds one single step)
    bytes_launch = BYTES_PER_NODE[args.form] * nodes      # state read + written once per launch
    hbm_gbs = bytes_launch / (launch_ms * 1e-3) / 1e9
    key = f"{args.form}_kbc{args.variant}_{n}" + ("_fused2" if spl == 2 else "")
    traffic = measured_traffic(key)
    kname = (f"k_step2<{args.form},KBC-{args.variant},64x{rows}>" if spl == 2
             else f"k_step<{args.form},KBC-{args.variant}>")
    if spl == 2 and args.variant == "B":
        # two steps per pass through HBM: the kernel is bound by vector
        # arithmetic, not by HBM
        flops_launch = FLOPS_PER_NODE_STEP[args.form] * nodes * spl
        achieved = flops_launch / (launch_ms * 1e-3) / 1e12
        peak = VECTOR_PEAK_TFLOPS[args.form]
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": kname,
                    "flops_kind": "FP32 operations of the compiled collision per node-step "
                                  f"({FLOPS_PER_NODE_STEP[args.form]}; FMA = 2), x {spl} steps x nodes per launch",
                    "peak_kind": "published FP32 vector peak, which assumes packed FP32; this library issues "
                                 "no packed FP32, so non-packed issue reaches at most half of it",
                    "steps_per_launch": spl, "algorithmic_flops_per_launch": flops_launch,
                    "algorithmic_bytes_per_launch": bytes_launch,
                    # the HBM side of the same launch: the state read and written once per launch
                    "hbm_GBs_per_launch": round(hbm_gbs, 1),
                    "hbm_frac_per_launch": round(hbm_gbs / HBM_PEAK_GBS, 4)}
        # the kernel's own limit: vector instructions issued (counted by the
        # profiler per node-step) against one instruction per lane and clock
        # on 256 CUs x 64 lanes at the nominal 2.4 GHz (packed FP32 is not
        # emitted, so the published FP32 peak above is twice what it can reach)
        ipn = measured_traffic(key, field="valu_instructions_per_node_step")
        if ipn:
            roofline["valu_instructions_per_node_step"] = ipn
            roofline["valu_issue_frac"] = round(ipn * nodes / (ms * 1e-3) / VALU_ISSUE_PEAK, 4)
    else:
        roofline = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                    "steps_per_launch": spl, "algorithmic_bytes_per_launch": bytes_launch}

    extras = {}
    want = set() if args.no_extras else set(args.extras.split(","))
    if want:
        # the same workload in the other storage forms and with the LBGK baseline
        for form in ("f16", "f64"):
            if form == args.form or "forms" not in want:
                continue
            s = make_sim(n, form, "kbc", args.variant, nu, seed, k0, dev)
            fs = s.fusion
            m, _ = time_steps(s, args.extra_steps, EXTRA_WARMUP)
            progress(f"{form}: {m:.4f} ms/step")
            del s
            torch.cuda.empty_cache()
            # HBM moves the state once per launch of fs steps
            extras[f"kbc{args.variant}_{form}"] = {
                "mlups": round(nodes / (m * 1e-3) / 1e6, 1), "ms_per_step": round(m, 4), "steps_per_launch": fs,
                "hbm_frac": round(BYTES_PER_NODE[form] * nodes / (fs * m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if "exact" in want:
        # the exact stabiliser: per-node Newton root of the entropy condition
        from paper_1507_02509_amd import inputs
        from paper_1507_02509_amd.sim import Sim, beta_from_nu
        ux, uy = inputs.spectral(n, k0, 0.05, seed=seed, device=dev)
        s = Sim(n, n, beta_from_nu(nu), collision="kbc", variant=args.variant, form=args.form,
                gamma_mode="exact", device=dev).init(ux, uy)
        del ux, uy
        fs = s.fusion
        m, _ = time_steps(s, args.extra_steps, EXTRA_WARMUP)
        progress(f"exact stabiliser: {m:.4f} ms/step")
        d = s.diagnostics()
        del s
        torch.cuda.empty_cache()
        extras[f"kbc{args.variant}_{args.form}_exact_gamma"] = {
            "mlups": round(nodes / (m * 1e-3) / 1e6, 1), "ms_per_step": round(m, 4), "steps_per_launch": fs,
            "over_estimate_time": round(m / ms, 3), "gamma_mean": d["gamma"]}
    if "lbgk" in want:
        s = make_sim(n, args.form, "lbgk", "A", nu, seed, k0, dev)
        fs = s.fusion
        m, _ = time_steps(s, args.extra_steps, EXTRA_WARMUP)
        del s
        torch.cuda.empty_cache()
        extras[f"lbgk_{args.form}"] = {"mlups": round(nodes / (m * 1e-3) / 1e6, 1), "ms_per_step": round(m, 4),
                                       "steps_per_launch": fs}
        extras["kbc_over_lbgk_time"] = round(ms / m, 3)
    if "copy" in want:
        # the copy reference: 2 x 1.2 GB read + write
        from paper_1507_02509_amd.sim import copy_probe
        a = torch.empty(300_000_000, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        copy_probe(b, a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            copy_probe(b, a)
        e1.record()
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1) / 10
        extras["copy_probe_GBs"] = round(2 * a.numel() * 4 / (cms * 1e-3) / 1e9, 1)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        extras["torch_copy_GBs"] = round(2 * a.numel() * 4 / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9, 1)
        # two streams read, one written (the adjoint step's pattern: state and
        # incoming adjoint in, outgoing adjoint out)
        c = torch.empty_like(a)
        torch.add(a, b, out=c)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            torch.add(a, b, out=c)
        e1.record()
        torch.cuda.synchronize()
        extras["torch_add_GBs"] = round(3 * a.numel() * 4 / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9, 1)
        del a, b, c
        torch.cuda.empty_cache()
    if "adjoint" in want:
        progress("adjoint kernel")
        ams = time_adjoint(n, nu, seed, k0, dev, steps=args.extra_steps)
        extras["adjoint_f32"] = {"mlups": round(nodes / (ams * 1e-3) / 1e6, 1), "ms_per_step": round(ams, 4),
                                 "bytes_per_node": 108,
                                 "hbm_frac": round(108 * nodes / (ams * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "adjoint_over_forward_step": round(ams / ms, 3),
                                 "traffic": measured_traffic(f"adjoint_f32_kbcB_{n}", section="adjoint")}
    if "rollout" in want:
        progress("rollout 512^2 x 2000")
        extras["rollout_512_2000_f32"] = time_c5(dev)
    if "ensemble" in want:
        progress("ensemble 256")
        extras["ensemble_256_f32"] = time_ensemble(dev, steps=args.extra_steps)
    if "slab" in want:
        progress("slab of an 8-way split")
        extras["slab_8way_f32"] = time_slab(dev, steps=args.extra_steps)
    if "accuracy" in want:
        progress("form errors")
        extras["accuracy"] = form_errors(n, nu, seed, k0, dev)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16": "f32 (f16 storage)", "f32": "f32", "f64": "f64"}[args.form],
        "data": "synthetic",
        "config": {"workload": workload, "nx": n, "ny": n, "collision": f"KBC-{args.variant}",
                   "form": f"{args.form}dev" if args.form != "f64" else "f64", "nu": nu, "seed": seed,
                   "k0": k0, "u_rms": 0.05, "init": "grad_cd"},
        "roofline": roofline,
        "wall_s_timed": round(wall, 3),
        "final_state": {"steps": args.warmup + args.steps,
                        "mass_drift_rel": (d_main["mass"] - d0["mass"]) / d0["mass"],
                        "E": d_main["E"], "Z": d_main["Z"], "gamma_mean": d_main["gamma"],
                        "n_nonfinite": d_main["n_nonfinite"]},
        "extras": extras,
    }
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(n, nu, seed, k0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
