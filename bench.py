"""Benchmark: energy + adjoint-gradient evaluations per second on one MI355X.

Workload (default): n = 28 qubits, complex64 state (2 GiB) with FP64
reductions, hardware-efficient ansatz with L = 6 layers of RY, RZ and a
linear CZ ladder (336 parameters), Hamiltonian of 20,000 Z-strings of weight
1-6 on a 16-community planted interaction graph (seed 0).  One step is one
energy + full gradient through ``GVEnergy`` (forward and backward); the
diagonal is built once before timing (it does not depend on the angles).

The JSON line also carries: the plain complex128 GPU path on the same
workload, the dominant kernel's achieved HBM bandwidth (algorithmic bytes per
launch over its HIP-event-timed average duration, taken inside the timed
region), the error against the stored oracle result, and the CPU oracle timed
on a bounded sample of the same evaluation.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", default="store", choices=["uncompute", "checkpoint", "recompute", "store"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="also time a 2 GiB device-to-device copy (the practical HBM ceiling, and "
                         "the reference kernel for scaling byte counters)")
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


def cpu_baseline(inst):
    """The oracle on host cores, on a bounded sample of one evaluation: one
    whole layer of the n=28 circuit forward (every RY, RZ and CZ gate), the
    reverse-sweep steps of the same layer, and the lambda = D psi product,
    each timed once; one evaluation runs L such layers each way (the
    theta-independent diagonal excluded, as on the GPU)."""
    import oracle
    n, L, ent = inst.n, inst.layers, inst.ent
    ng = oracle.num_gates(n, L, ent)
    per_layer = ng // L
    assert ng == L * per_layer
    dim = 1 << n
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
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": 1.0 / est, "unit": "evals/s", "cores": threads, "kind": "oracle",
        "sample": (f"complex128 oracle at n={n}: one full layer forward ({per_layer} gates, "
                   f"{t_f:.1f} s), its {per_layer} reverse-sweep steps ({t_b:.1f} s) and one "
                   f"lambda=D*psi product ({t_h:.1f} s), scaled to the {L} layers of one "
                   f"evaluation: est. {est:.1f} s/eval; diagonal build excluded"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this engine has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2607_02749_amd import gv, synth

    inst = synth.workload_n28()
    an = gv.Ansatz(inst.n, inst.layers, inst.ent)
    log("workload ready", inst.n, inst.layers, inst.num_terms)

    st = gv.State(inst.n, "c64", "fused", an, args.mode)
    t0 = time.perf_counter()
    h = gv.PauliSum(inst.n, inst.x, inst.z, inst.c).prepare(st)
    torch.cuda.synchronize()
    diag_ms = (time.perf_counter() - t0) * 1e3
    theta = torch.tensor(inst.theta, dtype=torch.float64, device=st.device, requires_grad=True)

    last = {}

    def step():
        E = gv.GVEnergy.apply(theta, st, h, an, None, args.mode)
        E.backward()
        last["E"] = E.detach()
        last["g"] = theta.grad
        theta.grad = None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    st.profile(True)
    st.profile_reset()
    wall, ev = time_steps(step, args.steps, torch)
    prof = st.profile_read()
    st.profile(False)
    log("timed", args.steps, "steps in", wall, "s")

    copy = None
    if args.copy_probe:
        src = torch.empty(1 << 31, dtype=torch.uint8, device=st.device)
        dst = torch.empty_like(src)
        src.fill_(1)
        dst.copy_(src)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 5
        copy = {"bytes": 2 * src.numel(), "ms": ms, "GBps": 2 * src.numel() / (ms * 1e-3) / 1e9}
        del src, dst

    value = args.steps / wall
    kinds = {k: v for k, v in prof.items() if v[0] > 0}
    dom = max(kinds, key=lambda k: kinds[k][1])
    n_l, ms_l, bytes_l = kinds[dom]
    avg_ms = ms_l / n_l
    achieved = (bytes_l / n_l) / (avg_ms * 1e-3) / 1e9
    kernel_names = {"backward_pass": "k_bwd_pass<float,12,4>", "forward_pass": "k_fwd_pass<float,12,4>",
                    "energy": "k_energy_diag<float>", "init": "k_init_state<float>"}
    breakdown = {k: {"launches_per_step": v[0] / args.steps, "ms_per_step": v[1] / args.steps,
                     "GBps": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None}
                 for k, v in kinds.items()}

    parity = None
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_n28.json")
    if os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        e_ref, g_ref = gold["energy"][0], np.array(gold["grad"])
        e = last["E"].item()
        g = last["g"].cpu().numpy()
        parity = {"energy_rel": abs(e - e_ref) / abs(e_ref),
                  "grad_rel_l2": float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))}

    plain = None
    if not args.no_plain:
        del st, h
        torch.cuda.empty_cache()
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

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        tr = json.load(open(tpath)).get(dom)
        if tr and tr.get("kernel_source_hash") == _kernel_hash():
            traffic = tr.get("bytes_per_launch")

    out = {
        "metric": "energy+adjoint-grad evals/s at n=28 c64 vs plain c128; HBM GB/s vs peak",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "n28_L6_czlinear_20000z", "n": inst.n, "layers": inst.layers,
                   "params": inst.num_params, "terms": inst.num_terms, "state": "complex64",
                   "reductions": "fp64", "gradient": "adjoint via torch.autograd.Function",
                   "grad_mode": args.mode, "seed": 0, "diag_build_ms": diag_ms,
                   "event_ms_per_step": ev / args.steps * 1e3},
        "roofline": {"bound": "hbm", "kernel": kernel_names.get(dom, dom), "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": bytes_l / n_l},
        "kernels": breakdown,
        "parity_vs_oracle": parity,
        "plain_c128": plain,
        "copy_probe": copy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("gv_fused.hip", "gv_device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2607_02749_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
