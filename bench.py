"""Benchmark: energy + adjoint-gradient evaluations per second on one MI355X.

Workload (default, ``--workload n28``): n = 28 qubits, complex64 state
(2 GiB) with FP64 reductions, hardware-efficient ansatz with L = 6 layers of
RY, RZ and a linear CZ ladder (336 parameters), Hamiltonian of 20,000
Z-strings of weight 1-6 on a 16-community planted interaction graph (seed 0).
One step is one energy + full gradient through ``GVEnergy`` (forward and
backward); the diagonal is built once before timing (it does not depend on
the angles).  The default gradient mode keeps every tile pass's output state
(``store``); ``--mode`` picks another.

The JSON line also carries: the dominant kernel's achieved HBM bandwidth
(algorithmic bytes per launch over its HIP-event-timed average duration on
the launch stream, inside the timed region) with the HBM bytes the hardware
counters measured for it, every kernel class's time, the error against the
stored oracle result, the plain complex128 GPU path on the same workload,
and the CPU oracle timed on a bounded sample of the same evaluation.

``--workload batch``: 256 uneven cluster instances (n in 12..20, L in 3..5,
50 n Z-strings + 5 n XX/YY terms each, restricted to the instance's
community) in one persistent kernel replayed from a HIP graph, with the
launch shape from the autotuner; instance evaluations per second.

``--workload n32``: n = 32 (32 GiB per complex64 state), L = 4, 50,000
Z-strings + 2,000 XX/YY/XZ/ZY terms in 64 qubit-wise-commuting groups; one
evaluation per gradient memory mode (uncompute, checkpoint, recompute, and
store when it fits), each with its device memory and time.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HBM_BYTES = 288 * 2**30

KERNELS = {
    "forward_pass": "k_fwd_load_pass<float,12,4>", "forward_pass2": "k_fwd2_load_pass<float,12,4>",
    "backward_pass": "k_bwd_pass<float,12,4>", "backward_ld": "k_bwd_ld_pass<float,12,4>",
    "backward_gf": "k_bwd_gf_pass<float,12,4>", "backward_gf_ld": "k_bwd_gf_ld_pass<float,12,4>",
    "turnaround": "k_turn_load_pass<float,12,4>", "first_layer": "k_layer0_grad<float,12,4>",
    "energy": "k_energy_diag<float>", "offdiag": "k_offdiag_pass<float,12,4,W>",
    "backward2": "k_bwd2_pass<float,12,4>",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="n28", choices=["n28", "n32", "batch", "pshift"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", default="store", choices=["uncompute", "checkpoint", "recompute", "store"])
    ap.add_argument("--no-copy-probe", action="store_true",
                    help="skip the streaming-kernel ceiling (hand-written read / write / copy / "
                         "read-modify-write kernels over 2 GiB buffers)")
    ap.add_argument("--stream-sweep", default=None,
                    help="write every streaming-kernel measurement of a wider sweep to this JSON file")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(step, k, torch):
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(k):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1000.0


def measure(inst, mode, steps, warmup, h=None):
    """Time `steps` evaluations (after `warmup`) of E and its gradient through
    GVEnergy in complex64; per-kernel-class HIP-event profile of the timed
    region.  h: a PauliSum already prepared for complex64 / fused."""
    import torch
    from paper_2607_02749_amd import gv
    an = gv.Ansatz(inst.n, inst.layers, inst.ent, inst.final_rotation)
    st = gv.State(inst.n, "c64", "fused", an, mode)
    diag_ms = None
    if h is None:
        # host: merge, split and group the terms; device: the FWHT diagonal
        # and the term tables (prepare waits for its stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = gv.PauliSum(inst.n, inst.x, inst.z, inst.c)
        t1 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        h.prepare(st)
        e1.record()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        diag_ms = {"host_ingest_ms": (t1 - t0) * 1e3, "prepare_wall_ms": (t2 - t1) * 1e3,
                   "prepare_stream_ms": e0.elapsed_time(e1)}
    theta = torch.tensor(inst.theta, dtype=torch.float64, device=st.device, requires_grad=True)
    last = {}

    def step():
        E = gv.GVEnergy.apply(theta, st, h, an, None, mode)
        E.backward()
        last["E"] = E.detach()
        last["g"] = theta.grad
        theta.grad = None

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st.profile(True)
    st.profile_reset()
    wall, ev = time_steps(step, steps, torch)
    prof = st.profile_read()
    st.profile(False)
    sb, wb = gv.query_sizes(an, "c64", "fused", mode)
    out = {"wall": wall, "ev": ev, "prof": prof, "E": last["E"].item(),
           "g": last["g"].cpu().numpy(), "state_bytes": sb, "work_bytes": wb,
           "h_bytes": h.device_bytes, "diag_ms": diag_ms}
    del st, theta, last
    torch.cuda.empty_cache()
    return out, h


def roofline(prof, steps):
    kinds = {k: v for k, v in prof.items() if v[0] > 0}
    dom = max(kinds, key=lambda k: kinds[k][1])
    n_l, ms_l, bytes_l = kinds[dom]
    avg_ms = ms_l / n_l
    achieved = (bytes_l / n_l) / (avg_ms * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        tr = json.load(open(tpath)).get(dom)
        if tr and tr.get("kernel_source_hash") == _kernel_hash():
            traffic = tr.get("bytes_per_launch")
    breakdown = {k: {"launches_per_step": v[0] / steps, "ms_per_step": v[1] / steps,
                     "GBps": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None}
                 for k, v in kinds.items()}
    roof = {"bound": "hbm", "kernel": KERNELS.get(dom, dom), "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": bytes_l / n_l}
    return roof, breakdown


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inst):
    """The oracle on host cores, on a bounded sample of one evaluation: one
    whole layer of the n=28 circuit forward (every RY, RZ and CZ gate), the
    reverse-sweep steps of the same layer, and the lambda = D psi product,
    each timed once with every host thread; one evaluation runs L such layers
    each way (the theta-independent diagonal excluded, as on the GPU).  Then
    the first 4 gates forward and back on one thread, scaled by the gate
    count of an evaluation."""
    import oracle
    n, L, ent = inst.n, inst.layers, inst.ent
    ng = oracle.num_gates(n, L, ent)
    per_layer = ng // L
    assert ng == L * per_layer
    dim = 1 << n
    threads = oracle.max_threads()
    phi = np.zeros(dim, np.complex128)
    phi[0] = 1.0
    grad = np.zeros(inst.num_params)
    t0 = time.perf_counter()
    oracle.apply_gates(n, L, ent, inst.theta, phi, 0, per_layer)
    t_f = time.perf_counter() - t0
    d = np.random.default_rng(0).normal(size=dim)
    t0 = time.perf_counter()
    lam = oracle.apply_h(n, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0), phi, d)
    oracle.inner(n, phi, lam)
    t_h = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.adjoint_gates(n, L, ent, inst.theta, phi, lam, grad, 0, per_layer)
    t_b = time.perf_counter() - t0
    est = L * (t_f + t_b) + t_h
    # one thread: 4 gates forward and their 4 reverse steps
    k = 4
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.apply_gates(n, L, ent, inst.theta, phi, 0, k)
        t_f1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.adjoint_gates(n, L, ent, inst.theta, phi, lam, grad, 0, k)
        t_b1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    est1 = ng * (t_f1 + t_b1) / k
    return {
        "value": 1.0 / est, "unit": "evals/s", "cores": threads, "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"complex128 oracle at n={n}, {threads} threads: one full layer forward "
                   f"({per_layer} gates, {t_f:.1f} s), its {per_layer} reverse-sweep steps "
                   f"({t_b:.1f} s) and one lambda=D*psi product ({t_h:.1f} s), scaled to the {L} "
                   f"layers of one evaluation: est. {est:.1f} s/eval; diagonal build excluded"),
        "one_thread": {"value": 1.0 / est1, "unit": "evals/s", "cores": 1,
                       "sample": (f"the first {k} gates forward ({t_f1:.1f} s) and back "
                                  f"({t_b1:.1f} s) on one thread, scaled to the {ng} gates "
                                  f"of an evaluation: est. {est1:.0f} s/eval")},
    }


def copy_probe(torch, gv, full=False):
    """Practical HBM ceiling: hand-written streaming kernels (gv_stream_probe)
    over 2 GiB buffers, for read, write, copy, read-modify-write (two streams
    read, one written back: the reverse passes' pattern) and triad, swept over
    bytes per lane, accesses in flight per lane, non-temporal hints and grid
    size; plus torch's own device copy.  Returns the best configuration per
    pattern (and every measurement when full)."""
    nb = 1 << 31
    bufs = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(3)]
    for b in bufs:
        b.fill_(0)
    moved = {"read": 1, "write": 1, "copy": 2, "rmw": 3, "triad": 3}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=3):
        fn()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    rows = []
    widths, unrolls, grids = (8, 16), (1, 2, 4, 8), (0, 1024, 2048, 4096)
    if not full:
        widths, unrolls, grids = (8, 16), (2, 4, 8), (0, 2048)
    for kind in ("read", "write", "copy", "rmw", "triad"):
        for w in widths:
            for u in unrolls:
                for nt in (0, 1):
                    for g in grids:
                        ms = timed(lambda: gv.stream_probe(kind, w, u, nt, g, bufs[0], bufs[1],
                                                           bufs[2], nb))
                        rows.append({"kind": kind, "width": w, "unroll": u, "nontemporal": nt,
                                     "grid": g, "ms": ms,
                                     "GBps": moved[kind] * nb / (ms * 1e-3) / 1e9})
    best = {}
    for r in rows:
        if r["kind"] not in best or r["GBps"] > best[r["kind"]]["GBps"]:
            best[r["kind"]] = r
    # the tile-pass layout: one amplitude (8 B) per lane, 16 in flight, runs of
    # 16 amplitudes 2^s apart (s = 12, 20: the second and third passes at n = 28)
    tiled = []
    if full:
        for kind in ("copy", "rmw"):
            for w in (8, 16):
                for shift in (0, 8, 10, 12, 14, 16, 17, 18, 19, 20, 21):
                    if shift and (nb // w) < (1 << (shift + 8)):
                        continue
                    for u, nt in ((16, 0), (16, 1), (4, 1)):
                        ms = timed(lambda: gv.stream_probe(kind, w, u, nt, 0, bufs[0], bufs[1],
                                                           bufs[2], nb, tile_shift=shift))
                        tiled.append({"kind": kind, "width": w, "unroll": u, "grid": 0,
                                      "nontemporal": nt, "tile_shift": shift, "ms": ms,
                                      "GBps": moved[kind] * nb / (ms * 1e-3) / 1e9})
    ms = timed(lambda: bufs[0].copy_(bufs[1]), 5)
    out = {"bytes_per_buffer": nb, "best": best,
           "torch_copy": {"ms": ms, "GBps": 2 * nb / (ms * 1e-3) / 1e9}}
    if full:
        out["all"] = rows
        out["tiled"] = tiled
    del bufs
    torch.cuda.empty_cache()
    return out


def bench_n28(args, torch, gv, synth):
    inst = synth.workload_n28()
    log("workload ready", inst.n, inst.layers, inst.num_terms)
    m, h = measure(inst, args.mode, args.steps, args.warmup)
    log("timed", args.steps, "steps in", m["wall"], "s")
    roof, breakdown = roofline(m["prof"], args.steps)
    copy = None
    if not args.no_copy_probe:
        copy = copy_probe(torch, gv, full=args.stream_sweep is not None)
        if args.stream_sweep:
            with open(args.stream_sweep, "w") as f:
                json.dump(copy, f, indent=1)
            copy.pop("all", None)
        log("copy probe", {k: round(v["GBps"]) for k, v in copy["best"].items()})

    parity = None
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_n28.json")
    if os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        e_ref, g_ref = gold["energy"][0], np.array(gold["grad"])
        parity = {"energy_rel": abs(m["E"] - e_ref) / abs(e_ref),
                  "grad_rel_l2": float(np.linalg.norm(m["g"] - g_ref) / np.linalg.norm(g_ref))}
    del h
    torch.cuda.empty_cache()

    plain = None
    if not args.no_plain:
        an = gv.Ansatz(inst.n, inst.layers, inst.ent)
        st2 = gv.State(inst.n, "c128", "plain", an)
        h2 = gv.PauliSum(inst.n, inst.x, inst.z, inst.c).prepare(st2)
        th2 = torch.tensor(inst.theta, dtype=torch.float64, device=st2.device)
        out2 = {}

        def step2():
            out2["e"], out2["g"] = gv.energy_grad(st2, h2, th2, an)

        step2()
        w2, _ = time_steps(step2, args.plain_steps, torch)
        plain = {"value": args.plain_steps / w2, "unit": "evals/s", "dtype": "c128",
                 "ms_per_step": w2 / args.plain_steps * 1e3, "engine": "plain (one kernel per gate)"}
        if parity is not None:
            plain["energy_rel"] = abs(out2["e"][0].item() - e_ref) / abs(e_ref)
            plain["grad_rel_l2"] = float(np.linalg.norm(out2["g"].cpu().numpy() - g_ref)
                                         / np.linalg.norm(g_ref))
        log("plain c128 done", plain["ms_per_step"], "ms/eval")
        del st2, h2

    cpu = None if args.no_cpu else cpu_baseline(inst)
    return {
        "metric": "energy+adjoint-grad evals/s at n=28 c64 vs plain c128; HBM GB/s vs peak",
        "value": args.steps / m["wall"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["wall"] / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "n28_L6_czlinear_20000z", "n": inst.n, "layers": inst.layers,
                   "params": inst.num_params, "terms": inst.num_terms, "state": "complex64",
                   "reductions": "fp64", "gradient": "adjoint via torch.autograd.Function",
                   "grad_mode": args.mode, "seed": 0, "diag_build_ms": m["diag_ms"],
                   "event_ms_per_step": m["ev"] / args.steps * 1e3,
                   "device_bytes": {"state": m["state_bytes"], "work": m["work_bytes"],
                                    "hamiltonian": m["h_bytes"]}},
        "roofline": roof,
        "kernels": breakdown,
        "parity_vs_oracle": parity,
        "plain_c128": plain,
        "copy_probe": copy,
        "cpu_baseline": cpu,
    }


def bench_n32(args, torch, gv, synth):
    """One evaluation per gradient memory mode at n = 32 (the workload does
    not fit the oracle: parity at this size is covered by the properties in
    tests/test_gpu_fullsize.py)."""
    inst = synth.workload_n32()
    log("workload ready", inst.n, inst.layers, inst.num_terms)
    an = gv.Ansatz(inst.n, inst.layers, inst.ent)
    h = None
    modes = {}
    e_ref = g_ref = None
    first = None
    for mode in ("uncompute", "checkpoint", "recompute", "store"):
        sb, wb = gv.query_sizes(an, "c64", "fused", mode)
        hb = h.device_bytes if h is not None else None
        need = sb + wb + (hb or (8 << inst.n))
        if need > HBM_BYTES - (8 << 30):
            modes[mode] = {"fits": False, "device_bytes": need}
            log(mode, "does not fit:", need / 2**30, "GiB")
            continue
        m, h = measure(inst, mode, args.steps, args.warmup, h)
        roof, breakdown = roofline(m["prof"], args.steps)
        if e_ref is None:
            e_ref, g_ref, first = m["E"], m["g"], m
        modes[mode] = {"fits": True, "ms_per_eval": m["wall"] / args.steps * 1e3,
                       "device_bytes": {"state": sb, "work": wb, "hamiltonian": m["h_bytes"]},
                       "energy_rel_vs_uncompute": abs(m["E"] - e_ref) / abs(e_ref),
                       "grad_rel_l2_vs_uncompute": float(np.linalg.norm(m["g"] - g_ref)
                                                         / np.linalg.norm(g_ref)),
                       "roofline": roof, "kernels": breakdown}
        log(mode, modes[mode]["ms_per_eval"], "ms/eval")
    u = modes["uncompute"]
    return {
        "metric": "energy+adjoint-grad evals/s at n=32 c64 per gradient memory mode",
        "value": 1e3 / u["ms_per_eval"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": u["ms_per_eval"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "n32_L4_czlinear_50000z_2000offdiag_64groups", "n": inst.n,
                   "layers": inst.layers, "params": inst.num_params, "terms": inst.num_terms,
                   "grad_mode": "uncompute", "diag_build_ms": first["diag_ms"]},
        "roofline": u["roofline"],
        "modes": modes,
        "cpu_baseline": None,
    }


def bench_batch(args, torch, gv, synth):
    """Config: 256 instances, complex64, one graph replay per step."""
    import oracle
    from paper_2607_02749_amd import autotune
    insts = synth.workload_batch(count=256)
    dev = torch.device("cuda", torch.cuda.current_device())
    items = []
    for inst in insts:
        an = gv.Ansatz(inst.n, inst.layers, inst.ent, inst.final_rotation)
        th = torch.tensor(inst.theta, dtype=torch.float64, device=dev)
        items.append((an, th, gv.PauliSum(inst.n, inst.x, inst.z, inst.c), inst.cluster_mask))
    tune = autotune.tune_batch(items, "c64")
    log("tuned", {k: tune[k] for k in ("blocks_per_cu", "order", "split_n", "lds_n", "ms", "cached")})
    b = gv.Batch(items, "c64", blocks_per_cu=tune["blocks_per_cu"], order=tune["order"],
                 split_n=tune["split_n"], lds_n=tune["lds_n"], graph=True)
    for _ in range(args.warmup):
        b.run()
    wall, ev = time_steps(b.run, args.steps, torch)
    # parity: the two smallest instances (persistent kernel) and the two
    # largest (whole-GPU passes) against the oracle (restricted gradient)
    by_size = sorted(range(len(insts)), key=lambda i: (insts[i].n, insts[i].layers))
    order = by_size[:2] + by_size[-2:]
    worst_e = worst_g = 0.0
    for i in order:
        inst = insts[i]
        mask = oracle.param_mask(inst.n, inst.layers, inst.cluster_mask)
        e_ref, g_ref = oracle.energy_grad(inst.n, inst.layers, inst.ent, inst.theta, inst.x,
                                          inst.z, inst.c, mask=mask)
        e = b.energies[i, 0].item()
        g = b.grads[i].cpu().numpy()
        worst_e = max(worst_e, abs(e - e_ref.real) / abs(e_ref.real))
        worst_g = max(worst_g, float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)))
    # algorithmic bytes of one batch: per instance and layer, the tile passes
    # (one per 12-bit tile set: 1 pass for n <= 12, 2 for n <= 20) read and
    # write psi forward and psi, lam backward, plus psi, D and lam for the
    # energy (layer 0 is generated)
    total = 0.0
    for inst in insts:
        A = 1 << inst.n
        npass = 1 if inst.n <= 12 else 2
        R = inst.layers + inst.final_rotation
        total += A * 8 * (2 * npass * (R - 1) + 4 * npass * R) + A * (8 + 8 + 8)
    ms = ev / args.steps * 1e3
    achieved = total / (ms * 1e-3) / 1e9
    return {
        "metric": "batched energy+restricted-grad instance evals/s (256 uneven instances, c64)",
        "value": len(insts) * args.steps / wall, "unit": "instance evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "batch256_n12-20_L3-5", "instances": len(insts),
                   "n_range": [min(x.n for x in insts), max(x.n for x in insts)],
                   "graph": True,
                   "tuning": {k: tune[k] for k in ("blocks_per_cu", "order", "split_n", "lds_n")},
                   "tuning_sweep_ms": tune.get("timings"),
                   "event_ms_per_step": ms},
        "roofline": {"bound": "hbm", "kernel": "k_batch<float>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "avg_launch_ms": ms,
                     "algorithmic_bytes_per_launch": total},
        "parity_vs_oracle": {"instances": order, "energy_rel_max": worst_e,
                             "grad_rel_l2_max": worst_g},
        "cpu_baseline": None,
    }


def bench_pshift(args, torch, gv, synth):
    """The paper's own gradient (Eq. 13): 2P shifted energy-only evaluations
    of one instance in one batched graph launch, beside the adjoint gradient
    (one reverse sweep) on the same instance; n = 16, L = 4 (P = 128),
    800 Z-strings + 80 XX/YY terms on a 3-community graph, complex64."""
    inst = synth.make_instance(16, 4, 800, 4, 3, seed=0, m_off=80, off_types=("XX", "YY"))
    an = gv.Ansatz(inst.n, inst.layers, inst.ent)
    dev = torch.device("cuda", torch.cuda.current_device())
    th = torch.tensor(inst.theta, dtype=torch.float64, device=dev)
    ps = gv.ParamShift(an, gv.PauliSum(inst.n, inst.x, inst.z, inst.c), precision="c64")
    for _ in range(args.warmup):
        ps(th)
    wall_ps, ev_ps = time_steps(lambda: ps(th), args.steps, torch)
    g_ps, _ = ps(th)
    st = gv.State(inst.n, "c64", "fused", an, "store")
    h = gv.PauliSum(inst.n, inst.x, inst.z, inst.c).prepare(st)
    out = {}

    def adj():
        out["e"], out["g"] = gv.energy_grad(st, h, th, an, None, "store")

    for _ in range(args.warmup):
        adj()
    wall_a, ev_a = time_steps(adj, args.steps, torch)
    g_ps = g_ps.cpu().numpy()
    g_a = out["g"].cpu().numpy()
    P = an.num_params
    return {
        "metric": "gradient evals/s: batched parameter shift (Eq. 13, 2P shifted circuits) vs adjoint",
        "value": args.steps / wall_ps, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_ps / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "pshift_n16_L4_800z_80offdiag", "n": inst.n, "layers": inst.layers,
                   "params": P, "shifted_circuits": 2 * P},
        "parameter_shift": {"gradients_per_s": args.steps / wall_ps,
                            "shifted_evals_per_s": 2 * P * args.steps / wall_ps,
                            "ms_per_gradient": ev_ps / args.steps * 1e3},
        "adjoint": {"gradients_per_s": args.steps / wall_a,
                    "ms_per_gradient": ev_a / args.steps * 1e3},
        "grad_rel_l2_shift_vs_adjoint": float(np.linalg.norm(g_ps - g_a) / np.linalg.norm(g_a)),
        "cpu_baseline": None,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this engine has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2607_02749_amd import gv, synth
    run = {"n28": bench_n28, "n32": bench_n32, "batch": bench_batch,
           "pshift": bench_pshift}[args.workload]
    out = run(args, torch, gv, synth)
    print(json.dumps(out))


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("gv_fused.hip", "gv_device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2607_02749_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
