"""Benchmark of the VQE hot path on one MI355X.

Workload (the batched potential-energy-surface scan): 100 bond lengths d in
[0.3, 3.0], integrals that are seeded smooth functions of d, the 4-qubit
model (2 spatial orbitals, HF |1100> + one DoubleExcitation) and the 8-qubit
model (4 spatial orbitals, all spin-conserving single and double
excitations from the HF state), each bond length optimised with Adam
(lr 0.01, 200 iterations, theta_0 = 0) on adjoint gradients (the
excitation gates and the Hamiltonians are real, so the library runs these
states on real f64 amplitudes; circuits with RX or RZ run complex128).
One step = one full scan of both qubit counts: 2 x 100 x 200 = 40,000
energy + gradient evaluations, the Hamiltonians resident on the device; the
two scans are independent and run on two HIP streams side by side.

Prints one JSON line.  Extra objects: `roofline` for the dominant kernel
(the persistent loop of the 8-qubit scan), `cpu_baseline` (the oracle on a
bounded sample of the same workload, one core and all cores, rank 0 only),
`setup` (host-side Hamiltonian build and upload per scan, outside the timed
region), `hea` (the hardware-efficient scaling sweep n = 12..26 with per-pass
HBM bandwidth at 26 qubits, where one state is 1 GiB, four times the last-level
cache), `large` (30 qubits energy + gradient, 32 qubits energy), `c1`, `qaoa`
and `served` (the mixed request stream at five arrival rates), each measured
outside the timed region.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6
ITERS = 200
BATCH = 100


def _progress(msg):
    """One progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hea", action="store_true")
    ap.add_argument("--hea-n", type=int, default=26, help="qubits of the per-pass bandwidth leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--no-qaoa", action="store_true")
    ap.add_argument("--scaling", type=str, default="12,16,20,24,26",
                    help="comma-separated qubit counts for the hardware-efficient scaling leg (L = n, 500 strings)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip 30-qubit energy + gradient and 32-qubit energy (L = 4, 2000 strings)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates the HBM byte "
                         "counters FETCH_SIZE / WRITE_SIZE of a profiler run) and exit")
    ap.add_argument("--served-requests", type=int, default=5000)
    ap.add_argument("--served-rates", type=str, default="0.25,0.5,1.0,1.5,2.0",
                    help="comma-separated multiples of the measured plain-path capacity")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-cores oracle leg (0: the host's cores, at most 16)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# algorithmic work per evaluation (counted from the problem, not the kernel)
# ---------------------------------------------------------------------------
GATE_FLOPS_PER_PAIR = {"RX": 12, "RY": 12, "RZ": 12, "H": 8, "X": 0, "CNOT": 0, "CZ": 0,
                       "SingleExcitation": 12, "DoubleExcitation": 12}
# active pairs of a gate on n qubits: 2^(n - number of pattern-fixed wires)
FIXED_WIRES = {"RX": 1, "RY": 1, "RZ": 1, "H": 1, "X": 1, "CNOT": 2, "CZ": 2, "SingleExcitation": 2,
               "DoubleExcitation": 4}


def eval_flops(spec, n_groups, complex_table, real_state=False):
    """Algorithmic FP64 flops of one energy + adjoint-gradient evaluation with
    H held as XOR-offset diagonals (lambda[b] = sum_f D_f[b] psi[b ^ f]; the
    diagonals are built once per Hamiltonian and reused by every iteration).

    Complex amplitudes: gates 12 flops per active amplitude pair for
    rotations, 8 for H, 0 for permutations; H psi 4 flops per amplitude per
    flip group (real diagonals; 8 when complex); E = Re<psi|lambda> 4 per
    amplitude; the reverse sweep the gates twice (psi and lambda) plus 7 flops
    per active pair of every parametric gate.  A state that stays real (real
    gate matrices, a real Hamiltonian) needs half of that for the gates, H psi
    and E, and 3 flops per pair for a gradient partial.
    """
    n = spec.n
    D = 1 << n
    fwd = 0
    grad = 0
    for k, p in zip(spec.kinds, spec.param_idx):
        pairs = D >> FIXED_WIRES[k]
        fwd += GATE_FLOPS_PER_PAIR[k] * pairs // (2 if real_state else 1)
        if p >= 0:
            grad += (3 if real_state else 7) * pairs
    hpsi = D * n_groups * (8 if complex_table else 4) // (2 if real_state else 1)
    energy = (2 if real_state else 4) * D
    return fwd + hpsi + energy + 2 * fwd + grad


def scope_table_flops(spec, n_terms):
    """The scope table's per-evaluation flop estimate for a small state:
    gates x 2^n amplitudes x 6 flops x 3 (forward, and the reverse sweep on psi
    and lambda) + 2 x terms x 2^n x 8 (the energy and H psi, term by term)."""
    D = 1 << spec.n
    return spec.n_gates * D * 6 * 3 + 2 * n_terms * D * 8


def _odd_y(x, z):
    """Terms whose phase i^{|x & z|} is imaginary (odd number of Y factors)."""
    return np.array([bin(int(a) & int(b)).count("1") % 2 == 1 for a, b in zip(x, z)], dtype=bool)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or None
    when none were taken or the kernel source changed since."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "gpus_requested": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    # the all-cores oracle leg runs in worker processes forked now, before
    # anything touches the GPU (they only ever run the CPU oracle)
    pool, workers = (None, 0) if args.no_cpu_baseline else _cpu_pool(args.cpu_workers)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)
        return

    import synth
    from paper_2601_09951_amd import vqe

    dev = torch.device("cuda:0")
    ctx = vqe.Context(0)

    # ---------------------------------------------------------------- setup
    ds = synth.bond_grid(BATCH)
    problems = []
    t0 = time.perf_counter()
    for n_orb, spec in ((2, synth.h2_circuit()), (4, synth.ucc_circuit(8, 2))):
        model = synth.smooth_integral_model(n_orb, seed=synth.MASTER_SEED)
        ints = [model.at(float(d)) for d in ds]
        # S0 on the device: the Jordan-Wigner map of Eq. (3) is built once per
        # orbital count; each scan evaluates H(d_i) for all bond lengths on the GPU
        fam = vqe.HamFamily(ctx, n_orb, BATCH)
        ints_dev = torch.tensor(vqe.HamFamily.pack(ints), dtype=torch.float64, device=dev)  # resident input
        hams = fam.members(BATCH)
        C = vqe.Circuit.from_spec(ctx, spec)
        theta = torch.zeros(BATCH, spec.n_params, dtype=torch.float64, device=dev)
        ws = vqe.workspace(ctx, C, hams, BATCH, 2)
        energies = torch.empty(BATCH, ITERS + 1, dtype=torch.float64, device=dev)
        problems.append(dict(n=spec.n, spec=spec, ints=ints, ints_dev=ints_dev, fam=fam, hams=hams, C=C,
                             theta=theta, ws=ws, energies=energies))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    # the two qubit counts are independent scans: each runs on its own HIP
    # stream (default priority), so the 4-qubit launch (100 workgroups) runs
    # beside the 8-qubit one (100 workgroups) on the other compute units;
    # the longer scan is issued first
    for p in problems:
        p["stream"] = torch.cuda.Stream(device=dev)
    order = sorted(range(len(problems)), key=lambda i: -problems[i]["n"])

    def one_scan(events=None):
        for i in order:
            p = problems[i]
            s = p["stream"]
            with torch.cuda.stream(s):
                p["fam"].set_integrals(p["ints_dev"])  # S0: H(d_i) for every bond length
                p["theta"].zero_()                      # theta_0 = 0
                if events is not None:
                    events[i][0].record(s)
                vqe.run(ctx, p["C"], p["hams"], p["theta"], ITERS, ws=p["ws"], energies=p["energies"])
                if events is not None:
                    events[i][1].record(s)

    _progress(f"setup {setup_s:.1f} s; warmup")
    for _ in range(args.warmup):
        one_scan()
    torch.cuda.synchronize()
    _progress("timed steps")

    K = args.steps
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in problems]
          for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        one_scan([ev[s][i] for i in range(len(problems))])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    evals = K * len(problems) * BATCH * ITERS
    value = evals / elapsed
    kernel_ms = {p["n"]: float(np.mean([ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(K)]))
                 for i, p in enumerate(problems)}

    # roofline of the dominant kernel: the persistent loop of the 8-qubit scan
    p8 = problems[1]
    x, z, c = p8["hams"][0].terms()
    n_groups = len(set(int(v) for v in x))
    complex_table = bool(np.any(_odd_y(x, z)))
    real_state = not complex_table and set(p8["spec"].kinds) <= synth.REAL_KINDS
    flops_eval = eval_flops(p8["spec"], n_groups, complex_table, real_state)
    flops_launch = flops_eval * BATCH * ITERS
    achieved = flops_launch / (kernel_ms[8] * 1e-3) / 1e12
    flops_scope = scope_table_flops(p8["spec"], len(c))
    achieved_scope = flops_scope * BATCH * ITERS / (kernel_ms[8] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_small_fast, 8 qubits (one workgroup of 320 threads per instance: a gate "
                                          "wave and four H psi waves; 100 instances x 200 steps in one launch; the "
                                          "event interval also holds the weight refresh, < 0.2 %)",
                "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 5),
                "traffic": measured_traffic("k_small_fast"),
                "flops_per_eval": flops_eval,
                "flops_count": "grouped: H held as XOR-offset diagonals, active pairs only (eval_flops)"
                               + ("; real amplitudes (real gates, real Hamiltonian)" if real_state else ""),
                "evals_per_launch": BATCH * ITERS, "kernel_ms": round(kernel_ms[8], 4),
                "scope_table_count": {"flops_per_eval": flops_scope, "achieved": round(achieved_scope, 4),
                                      "frac": round(achieved_scope / FP64_PEAK_TFLOPS, 5),
                                      "formula": "gates x 2^n x 6 x 3 + 2 x terms x 2^n x 8"}}

    final_e = {p["n"]: p["energies"][:, -1].cpu().numpy() for p in problems}
    out = {
        "metric": "VQE energy+grad evals/s (batched PES scan, 4q + 8q)",
        "value": round(value, 1),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched PES scan: 100 bond lengths x 200 Adam steps, 4-qubit H2-like "
                               "(15 terms) and 8-qubit all-excitations (UCC) models in f64 (real excitation gates and real Hamiltonians keep the state real; other circuits run complex128); each step "
                               "builds H(d_i) on the device (Jordan-Wigner map) and runs the full loop",
                   "global_batch": BATCH, "iterations": ITERS, "qubits": [4, 8],
                   "evals_per_step": len(problems) * BATCH * ITERS},
        "kernel_ms": {f"{k}q": round(v, 4) for k, v in kernel_ms.items()},
        "setup": {"seconds": round(setup_s, 3),
                  "what": "once per orbital count (outside timing): symbolic Jordan-Wigner map, circuit and "
                          "Hamiltonian plans, workspace; each timed step builds all 200 H(d_i) on the device"},
        "roofline": roofline,
        "pes_min_energy": {f"{k}q": round(float(np.min(v)), 10) for k, v in final_e.items()},
    }

    # -------------------------------------------------- large-state HEA
    _progress(f"scan: {value:.0f} evals/s")
    if not args.no_hea:
        out["hea"] = hea_measure(ctx, vqe, synth, torch, args.hea_n)
        _progress("hea done")
        if args.scaling:
            out["hea"]["scaling"] = []
            for v in args.scaling.split(","):
                out["hea"]["scaling"].append(scaling_measure(ctx, vqe, synth, torch, int(v)))
                _progress(f"scaling n={v} done")

    # -------------------------------------------------- C1: plain vs batched
    if not args.no_c1:
        out["c1"] = c1_measure(ctx, vqe, synth, torch)
        _progress("c1 done")
    if not args.no_qaoa:
        out["qaoa"] = qaoa_measure(ctx, vqe, synth, torch, 24, 4)
        _progress("qaoa done")
    if not args.no_large:
        out["large"] = large_measure(ctx, vqe, synth, torch)
        _progress("large done")

    # -------------------------------------------------- served stream
    if not args.no_served:
        out["served"] = served_measure(ctx, args.served_requests,
                                       tuple(float(x) for x in args.served_rates.split(",")))
        _progress("served done")

    # -------------------------------------------------- CPU baseline
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problems, args.cpu_seconds, pool, workers)
        pool.close()
        pool.join()

    print(json.dumps(out), flush=True)


def fused_pass_flops(ctx, vqe, C, n):
    """FP64 flops of one evaluation's fused passes, from the plan (FMA = 2):
    forward, per stage and chain (register chains and the exchanged qubit) a
    2x2 on every pair, 16 flops per amplitude, and 6 per amplitude for each
    parity phase; adjoint, the 2x2 on both states (32 per amplitude) plus,
    for a chain with parametric gates, its three pair sums (12), and for a
    phase 12 (both states) plus 4 when it is parametric.  Returns (forward
    flops, adjoint flops) per evaluation."""
    out = []
    for rev in (False, True):
        passes, _, fst, _, soff, _, sinfo, fph = vqe.circuit_plan(ctx, C, reverse=rev, stages="fused")
        flops = 0.0
        for p in passes:
            for s in range(int(p["fstage_begin"]), int(p["fstage_begin"]) + int(p["fstage_count"])):
                f = fst[s]
                nb = int(f["nb"])
                chains = list(range(int(f["na"]))) + ([nb] if int(f["xbit"]) else [])
                for j in chains:
                    sl = int(f["slot"]) + j
                    par = any(int(sinfo[e]) >= 16 for e in range(int(soff[sl]), int(soff[sl + 1])))
                    flops += (32 + (12 if par else 0)) if rev else 16
                for q in range(int(f["phase_begin"]), int(f["phase_begin"]) + int(f["phase_count"])):
                    flops += (12 + (4 if int(fph[q]["info"]) >= 16 else 0)) if rev else 6
        out.append(flops * (1 << n))
    return out[0], out[1]


def hea_measure(ctx, vqe, synth, torch, n):
    """Energy + adjoint gradient of the hardware-efficient ansatz (L = n
    layers, 500 random Pauli strings) at n qubits, then the same calls again
    with the library's kernel timing on (HIP events around every launch, on
    its own stream): per kernel class the average duration, the algorithmic
    HBM bytes per launch and their ratio against the 8 TB/s peak.  At 26
    qubits one state is 1 GiB, four times the 256 MB last-level cache, so the
    bytes come from HBM."""
    dev = torch.device("cuda:0")
    spec = synth.hea_circuit(n, n)
    ham = synth.random_pauli_sum(n, 500, seed=synth.MASTER_SEED + n)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th = torch.tensor(synth.uniform_thetas(spec.n_params, 1, seed=synth.MASTER_SEED + n), device=dev)
    ws = vqe.workspace(ctx, C, H, 1, 1)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(1, spec.n_params, dtype=torch.float64, device=dev)
    vqe.energy_grad(ctx, C, H, th, ws=ws, out_e=e, out_g=g)
    vqe.energy(ctx, C, H, th, ws=ws, out=e)
    torch.cuda.synchronize()
    reps = 2
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(reps):
        vqe.energy_grad(ctx, C, H, th, ws=ws, out_e=e, out_g=g)
    s1.record()
    torch.cuda.synchronize()
    ms_eval = s0.elapsed_time(s1) / reps
    s0.record()
    for _ in range(reps):
        vqe.energy(ctx, C, H, th, ws=ws, out=e)
    s1.record()
    torch.cuda.synchronize()
    ms_energy = s0.elapsed_time(s1) / reps
    ctx.profile(reset=True)
    ctx.set_profiling(True)
    for _ in range(reps):
        vqe.energy_grad(ctx, C, H, th, ws=ws, out_e=e, out_g=g)
        vqe.energy(ctx, C, H, th, ws=ws, out=e)
    prof = ctx.profile(reset=True)
    ctx.set_profiling(False)
    kernels = {}
    for name, r in sorted(prof.items()):
        if r["bytes"] <= 0:
            continue
        gbps = r["bytes"] / (r["ms"] * 1e-3) / 1e9
        kernels[name] = {"launches_per_eval": r["launches"] // reps, "avg_us": round(r["ms"] / r["launches"] * 1e3, 2),
                         "bytes_per_launch": int(r["bytes"] / r["launches"]), "GBps": round(gbps, 1),
                         "frac_of_hbm": round(gbps / HBM_PEAK_GBPS, 4)}
        # HBM bytes per launch from the committed counter runs (26 qubits, the
        # same kernel source), beside the algorithmic bytes
        base = {"k_pauli_sweep (expectation)": "k_pauli_sweep"}.get(name, name)
        tb = measured_traffic(base) if n == 26 and base in ("k_forward_fused", "k_reverse_fused", "k_hpsi_gather",
                                                             "k_pauli_sweep") else None
        kernels[name]["traffic_bytes_per_launch"] = tb
        kernels[name]["traffic_over_algorithmic"] = round(tb / (r["bytes"] / r["launches"]), 4) if tb else None
    # FP64 rate of the fused passes (their other bound: arithmetic per
    # amplitude with the tile held on chip)
    ff, fr = fused_pass_flops(ctx, vqe, C, n)
    for name, fl in (("k_forward_fused", ff), ("k_reverse_fused", fr)):
        if name in kernels:
            kk = kernels[name]
            per_launch = fl / (kk["launches_per_eval"] / (2 if name == "k_forward_fused" else 1))
            kk["fp64_flops_per_launch"] = int(per_launch)
            kk["fp64_tflops"] = round(per_launch / (kk["avg_us"] * 1e-6) / 1e12, 2)
            kk["frac_of_fp64"] = round(kk["fp64_tflops"] / FP64_PEAK_TFLOPS, 4)
    passes, _ = vqe.circuit_plan(ctx, C)
    pl = vqe.hamiltonian_plan(ctx, H, 1, False)
    del ws
    torch.cuda.empty_cache()
    return {"n": n, "layers": n, "gates": spec.n_gates, "params": spec.n_params, "terms": 500,
            "flip_groups": int(H.n_groups), "state_GiB": round((16 << n) / 2 ** 30, 3),
            "ms_per_energy_grad": round(ms_eval, 3), "ms_per_energy": round(ms_energy, 3),
            "forward_passes": int(len(passes)), "expect_sweeps": int(len(pl["sweeps"])),
            "kernels": kernels,
            "timing": "HIP events around each launch on its stream (library kernel timing), "
                      f"{reps} energy + gradient and {reps} energy evaluations; bytes = algorithmic "
                      "(forward pass 32 B, adjoint pass 64 B, expectation sweep 16 B, H psi sweep "
                      "32 / 48 B per amplitude)"}


def qaoa_measure(ctx, vqe, synth, torch, n, layers):
    """QAOA MaxCut (the diagonal-only Hamiltonian path): energy + adjoint
    gradient on a ring of n vertices with n / 2 random chords, `layers`
    layers (2 shared parameters each)."""
    dev = torch.device("cuda:0")
    edges = synth.ring_graph(n, n // 2, seed=synth.MASTER_SEED + n)
    spec = synth.qaoa_circuit(n, edges, layers)
    ham = synth.maxcut_hamiltonian(n, edges)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th = torch.tensor(synth.uniform_thetas(spec.n_params, 1, seed=synth.MASTER_SEED + n), device=dev)
    ws = vqe.workspace(ctx, C, H, 1, 1)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(1, spec.n_params, dtype=torch.float64, device=dev)
    vqe.energy_grad(ctx, C, H, th, ws=ws, out_e=e, out_g=g)
    torch.cuda.synchronize()
    reps = 3
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(reps):
        vqe.energy_grad(ctx, C, H, th, ws=ws, out_e=e, out_g=g)
    s1.record()
    torch.cuda.synchronize()
    passes = vqe.circuit_plan(ctx, C)[0]
    rpasses = vqe.circuit_plan(ctx, C, reverse=True)[0]
    return {"n": n, "layers": layers, "edges": len(edges), "gates": spec.n_gates, "params": spec.n_params,
            "terms": len(edges), "flip_groups": int(H.n_groups), "forward_passes": int(len(passes)),
            "adjoint_passes": int(len(rpasses)), "ms_per_energy_grad": round(s0.elapsed_time(s1) / reps, 3)}


def c1_measure(ctx, vqe, synth, torch):
    """The 4-qubit H2-like model: 100 energy-only theta points and 50
    gradient-descent steps (lr 0.2), once one instance per launch sequence with
    a host synchronisation per evaluation (the plain path), once batched /
    persistent."""
    dev = torch.device("cuda:0")
    ints = synth.random_integrals(2, seed=synth.MASTER_SEED)
    C = vqe.Circuit.from_spec(ctx, synth.h2_circuit())
    H = vqe.Hamiltonian.from_integrals(ctx, ints.h1, ints.h2)
    thetas = synth.theta_grid(100)
    ws = vqe.workspace(ctx, C, H, 1, 0)
    wsg = vqe.workspace(ctx, C, H, 1, 1)
    for _ in range(3):
        vqe.energy(ctx, C, H, torch.zeros(1, 1, dtype=torch.float64, device=dev), ws=ws).item()
    t0 = time.perf_counter()
    for t in thetas:
        vqe.energy(ctx, C, H, torch.full((1, 1), float(t), dtype=torch.float64, device=dev), ws=ws).item()
    plain_points = time.perf_counter() - t0
    th_all = torch.tensor(thetas[:, None], dtype=torch.float64, device=dev)
    wsb = vqe.workspace(ctx, C, H, len(thetas), 0)
    vqe.energy(ctx, C, H, th_all, ws=wsb)
    torch.cuda.synchronize()
    reps = []
    for _ in range(11):  # one call for all 100 points, result on the host; median of 11
        t0 = time.perf_counter()
        vqe.energy(ctx, C, H, th_all, ws=wsb).cpu()
        reps.append(time.perf_counter() - t0)
    batched_points = sorted(reps)[len(reps) // 2]
    # 50 GD steps: plain = energy_grad + host update per step
    th = 0.0
    t0 = time.perf_counter()
    for _ in range(50):
        e, g = vqe.energy_grad(ctx, C, H, torch.full((1, 1), th, dtype=torch.float64, device=dev), ws=wsg)
        th -= 0.2 * g.item()
    plain_gd = time.perf_counter() - t0
    tt = torch.zeros(1, 1, dtype=torch.float64, device=dev)
    vqe.run(ctx, C, H, tt, 50, optimizer="gd", lr=0.2)
    torch.cuda.synchronize()
    tt.zero_()
    t0 = time.perf_counter()
    traj = vqe.run(ctx, C, H, tt, 50, optimizer="gd", lr=0.2).cpu()
    persistent_gd = time.perf_counter() - t0
    return {"theta_points": 100, "plain_evals_per_s": round(100 / plain_points, 1),
            "batched_evals_per_s": round(100 / batched_points, 1),
            "gd_steps": 50, "plain_gd_ms_per_step": round(plain_gd / 50 * 1e3, 4),
            "persistent_gd_ms_per_step": round(persistent_gd / 50 * 1e3, 4),
            "gd_final_energy": round(float(traj[0, -1]), 12)}


def _hea_eval(ctx, vqe, synth, torch, n, layers, terms, batch, want_grad, reps=3, graphs=True, tune=False, warm=2):
    """ms per energy (+ gradient) evaluation of the hardware-efficient ansatz:
    two untimed calls (plans; with graphs on, the capture), then `reps` timed
    calls between events.  tune: vqe_autotune first (its choice is used and
    returned)."""
    dev = torch.device("cuda:0")
    spec = synth.hea_circuit(n, layers)
    ham = synth.random_pauli_sum(n, terms, seed=synth.MASTER_SEED + n)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th = torch.tensor(synth.uniform_thetas(spec.n_params, batch, seed=synth.MASTER_SEED + n), device=dev)
    ctx.set_graphs(graphs)
    tuned = vqe.autotune(ctx, C, H, th, want_grad=want_grad) if tune else None
    ws = vqe.workspace(ctx, C, H, batch, 1 if want_grad else 0)
    call = (lambda: vqe.energy_grad(ctx, C, H, th, ws=ws)) if want_grad else (lambda: vqe.energy(ctx, C, H, th, ws=ws))
    for _ in range(warm):
        call()
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(reps):
        call()
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / reps
    ctx.clear_tuning()
    ctx.set_graphs(False)  # the library default
    del ws
    torch.cuda.empty_cache()
    return ms, spec, H, tuned


def scaling_measure(ctx, vqe, synth, torch, n):
    """Energy + adjoint gradient of the hardware-efficient ansatz, L = n layers,
    500 random strings: one instance per call, and batches of 8 and 32 where
    the states are small; each eager (one launch per kernel), replayed from a
    captured graph, and with the autotuner's tiles / batch tile (plus graphs)."""
    reps = 2 if n >= 24 else 5
    out = {"n": n}
    for B in ((1, 8, 32) if n <= 20 else (1,)):
        row = {}
        ms_e, spec, H, _ = _hea_eval(ctx, vqe, synth, torch, n, n, 500, B, True, reps=reps, graphs=False)
        ms_g, _, _, _ = _hea_eval(ctx, vqe, synth, torch, n, n, 500, B, True, reps=reps, graphs=True)
        row["eager_evals_per_s"] = round(B / (ms_e * 1e-3), 2)
        row["graph_evals_per_s"] = round(B / (ms_g * 1e-3), 2)
        if n <= 24:
            ms_t, _, _, tuned = _hea_eval(ctx, vqe, synth, torch, n, n, 500, B, True, reps=reps, graphs=True,
                                          tune=True)
            row["tuned_evals_per_s"] = round(B / (ms_t * 1e-3), 2)
            row["tuned"] = {k: tuned[k] for k in ("k_fwd", "k_rev", "c_low", "wg_max", "batch_tile", "candidates")}
        out[f"batch{B}"] = row
    out.update({"gates": spec.n_gates, "params": spec.n_params, "flip_groups": int(H.n_groups),
                "ms_per_energy_grad": round(1e3 / out["batch1"]["graph_evals_per_s"], 3)})
    return out


def large_measure(ctx, vqe, synth, torch):
    """30 qubits energy + gradient (two resident 16 GiB states) and 32 qubits
    energy only (one 64 GiB state); hardware-efficient ansatz with 4 layers,
    2000 random strings."""
    ms30, spec30, H30, _ = _hea_eval(ctx, vqe, synth, torch, 30, 4, 2000, 1, True, reps=1, graphs=False, warm=1)
    ms32, spec32, H32, _ = _hea_eval(ctx, vqe, synth, torch, 32, 4, 2000, 1, False, reps=1, graphs=False, warm=1)
    return {"n30_energy_grad_s": round(ms30 * 1e-3, 3), "n30_flip_groups": int(H30.n_groups),
            "n32_energy_s": round(ms32 * 1e-3, 3), "n32_flip_groups": int(H32.n_groups),
            "n32_state_GiB": 64}


def served_measure(ctx, count, rates=(1.0,)):
    """The served mix (n in 4..24 with weights 40/25/15/10/6/4 %, energy-only or
    energy + gradient 50/50): the plain path (arrival order, one request per
    launch sequence, host sync each) sets the capacity; the continuous-batching
    server then serves Poisson arrivals at multiples of that capacity."""
    import synth
    from paper_2601_09951_amd import serve
    reqs = synth.served_requests(count, 1000.0, seed=synth.MASTER_SEED + 5)
    serve.run_plain(ctx, reqs[:20], realtime=False)  # warm plans and code objects
    t0 = time.perf_counter()
    plain = serve.run_plain(ctx, reqs, realtime=False)
    plain_wall = time.perf_counter() - t0
    capacity = count / plain_wall
    out = {"requests": count, "plain_capacity_evals_per_s": round(capacity, 1), "rates": []}
    ex = serve.LibvqeExecutor(ctx)
    srv = serve.Server(ex, mem_budget=32 << 30, max_batch=128)
    srv.run(synth.served_requests(40, 1000.0, seed=synth.MASTER_SEED + 6), realtime=False)  # warm
    for mult in rates:
        rate = mult * capacity
        rq = synth.served_requests(count, rate, seed=synth.MASTER_SEED + 5)
        res = srv.run(rq)
        s = serve.latency_summary(res)
        # the same arrival trace through the plain path
        pres = serve.run_plain(ctx, rq)
        ps = serve.latency_summary(pres)
        out["rates"].append({"rate_x_plain_capacity": mult, "offered_per_s": round(rate, 1),
                             "served": s, "plain": {k: ps[k] for k in ("p50_ms", "p99_ms", "evals_per_s")}})
    ex.close()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _cpu_pool(requested):
    """Worker processes for the all-cores oracle leg, forked before the GPU is
    initialised (each runs the oracle on one thread)."""
    import multiprocessing as mp
    import oracle
    oracle.lib()  # built once here, not by every worker
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = requested or max(1, min(16, avail))
    return mp.get_context("fork").Pool(workers), workers


def _oracle_bond(task):
    """One bond length on the oracle: Hamiltonian build and the Adam loop."""
    spec, ints, iters = task
    import oracle
    from oracle import fermion
    from threadpoolctl import threadpool_limits
    oracle.set_threads(1)
    threadpool_limits(1)  # one core per bond: numpy's BLAS in the Hamiltonian build too
    t0 = time.perf_counter()
    ho = fermion.qubit_hamiltonian(ints)
    e, _ = oracle.vqe_run(spec, ho, np.zeros(spec.n_params), iters)
    return time.perf_counter() - t0, float(e[-1])


def cpu_baseline(problems, budget_s, pool, workers):
    """The oracle (plain FP64 C for the loop) on a bounded sample of the same
    scan: the first bond lengths of each qubit count, each with its
    Hamiltonian build (the oracle's dense Jordan-Wigner construction, as the
    GPU step builds H(d_i) too) and 200 Adam steps on adjoint gradients.

    (i) one core: bond lengths one after another, about budget_s / 2 seconds
    per qubit count; (ii) all cores: bond lengths in parallel, one oracle
    process per core (the bond lengths are independent, so this is the
    paper's MPI-over-bond-lengths pattern), at least one bond per worker.
    Rates are scaled to the full scan; both runs compute the same final
    energies bit for bit (checked)."""
    import oracle
    oracle.set_threads(1)
    done, spent, final = {}, {}, {}
    for p in problems:
        n = p["n"]
        done[n], spent[n], final[n] = 0, 0.0, []
        wall0 = time.perf_counter()
        while done[n] < BATCH and (done[n] == 0 or time.perf_counter() - wall0 < budget_s / 2):
            dt, ef = _oracle_bond((p["spec"], p["ints"][done[n]], ITERS))
            spent[n] += dt
            final[n].append(ef)
            done[n] += 1
    scan_s = sum(spent[n] / done[n] * BATCH for n in spent)
    evals = len(spent) * BATCH * ITERS
    one = {"value": round(evals / scan_s, 1), "cores": 1,
           "per_qubit_evals_per_s": {f"{n}q": round(done[n] * ITERS / spent[n], 1) for n in sorted(spent)},
           "sample": " and ".join(f"{done[n]} x {n}q" for n in sorted(done)) + " bond lengths"}
    par, agree = {}, 0.0
    for p in problems:
        n = p["n"]
        cnt = min(BATCH, max(workers, done[n]))
        t0 = time.perf_counter()
        res = pool.map(_oracle_bond, [(p["spec"], p["ints"][i], ITERS) for i in range(cnt)], chunksize=1)
        par[n] = (cnt, time.perf_counter() - t0)
        for i, ef in enumerate(final[n]):
            agree = max(agree, abs(res[i][1] - ef))
    assert agree <= 1e-12, f"all-cores oracle run disagrees with the one-core run by {agree}"
    scan_par = sum(par[n][1] / par[n][0] * BATCH for n in par)
    return {"value": round(evals / scan_par, 1), "unit": "evals/s", "cores": workers, "kind": "oracle",
            "sample": " and ".join(f"{par[n][0]} x {n}q" for n in sorted(par))
                      + f" bond lengths on {workers} worker processes (one oracle thread each), each bond with "
                      f"its Hamiltonian build and {ITERS} Adam steps (adjoint gradients); wall time scaled to "
                      f"the full 2 x {BATCH}-bond scan",
            "per_qubit_evals_per_s": {f"{n}q": round(par[n][0] * ITERS / par[n][1], 1) for n in sorted(par)},
            "host": {"nproc": os.cpu_count(), "cpu_model": _cpu_model(), "threads_used": workers},
            "one_core": one, "max_final_energy_diff_vs_one_core": agree}


if __name__ == "__main__":
    main()
