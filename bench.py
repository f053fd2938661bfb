"""Benchmark: one step = the whole hot path on the 30-qubit layered circuit.

Workload (the metric's configuration): n = 30 qubits, complex128 state
(16 GiB), 20 layers of Haar-random U(2) on every qubit followed by CZ on
alternating nearest-neighbour bricks (890 gates, seed 2), then the
amplitudes of 4096 seeded bitstrings (seed 1002) and the FP64 norm.

A step = init |0...0> + every gate (planner mode, default "tile": on-chip
tile passes) + amplitude read-out + norm, inputs resident in HBM.  The value
is gate-updates/s = 890 / step time (a gate-update is one logical gate
applied to all 2^30 amplitudes).  The roofline figure is for the dominant
kernel (the tile pass): algorithmic bytes per pass (read + write of the whole
state, 32 GiB) divided by its device duration from HIP events recorded on the
state's stream around every pass of the timed steps.

usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--mode tile]
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gate-updates/s and achieved HBM GB/s per gate pass (fraction of peak), 1 GPU"
HBM_PEAK_GBPS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 FP64 FMA lanes x 2 flops x 2.4 GHz
FP32_MFMA_PEAK_TFLOPS = 157.3   # dense FP32 matrix-core peak (the in-tile 8x8 ops of C64 passes)
FUSE_K_C128 = 5                 # fused block width of the fused comparison step



def gate_flops_per_amp(gates, W) -> float:
    """Algorithmic flops per state amplitude of a gate list: a dense 2x2
    complex product is 14 flops per amplitude; diagonal and controlled gates
    touch a half or a quarter of the amplitudes; CNOT only moves data."""
    per = {W.OP_H: 14.0, W.OP_X: 14.0, W.OP_Y: 14.0, W.OP_U: 14.0, W.OP_Z: 3.0, W.OP_S: 3.0,
           W.OP_T: 3.0, W.OP_CNOT: 0.0, W.OP_CZ: 0.5, W.OP_CP: 1.5}
    return float(sum(per[int(op)] for op in gates["op"]))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _oracle_run(psi, n, gates, threads, budget_s):
    """Applies gate records with the oracle until the budget is spent and
    returns (gates done, seconds).  With threads > 1 the state is cut into
    2^a contiguous sub-vectors (2^a <= threads) that every gate whose qubits
    lie below n - a acts on independently, one worker thread each (numpy
    releases the interpreter lock inside its array loops); the computation
    per sub-vector is the oracle's own."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import statevector as sv
    a = max(0, int(threads).bit_length() - 1)
    chunks = psi.reshape(1 << a, -1)
    done = 0
    t1 = time.perf_counter()
    with ThreadPoolExecutor(max(1, 1 << a)) as pool:
        for rec in gates:
            qs = [int(rec["q0"])] + ([int(rec["q1"])] if int(rec["q1"]) >= 0 else [])
            if a == 0 or max(qs) >= n - a:
                sv.apply_record(psi, n, rec)
            else:
                list(pool.map(lambda c: sv.apply_record(chunks[c], n - a, rec), range(1 << a)))
            done += 1
            if time.perf_counter() - t1 > budget_s:
                break
    return done, time.perf_counter() - t1


def cpu_baseline(n, gates, budget_s):
    """Times the FP64 CPU oracle on the same circuit at full size: the first
    gates of the circuit on the 2^30-amplitude state, on every host core and
    on one, half the budget each."""
    from oracle import statevector as sv
    cores = max(1, min(os.cpu_count() or 1, 64))
    t0 = time.perf_counter()
    psi = sv.init_state(n)
    t_init = time.perf_counter() - t0
    done_all, el_all = _oracle_run(psi, n, gates, cores, budget_s / 2)
    used = 1 << (cores.bit_length() - 1)
    psi = sv.init_state(n)
    done_one, el_one = _oracle_run(psi, n, gates, 1, budget_s / 2)
    del psi
    host = f"host: {cpu_model()}, {os.cpu_count()} logical CPUs"
    return {"value": done_all / el_all, "unit": "gate-updates/s", "cores": used, "kind": "oracle",
            "sample": (f"first {done_all} of {len(gates)} gates of the same n={n} circuit on the full "
                       f"FP64 state, {used} threads over {used} independent sub-vectors (numpy), "
                       f"{el_all:.1f} s; init {t_init:.1f} s; {host}"),
            "single_core": {"value": done_one / el_one, "unit": "gate-updates/s", "cores": 1,
                            "sample": f"first {done_one} gates on one thread, {el_one:.1f} s"}}


TILE_SOURCES = ("k_tile.hip", "tile_ops.hpp", "juqcs_internal.hpp")
TUNING_RECORD = os.path.join(ROOT, "paper_1912_03243_amd", "tuning_mi355x.json")


def sources_sha256(names):
    """One digest over the kernel's source files, in the given order."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1912_03243_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_for(names):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), used
    only while the kernel's sources are unchanged since the measurement."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("source_sha256") == sources_sha256(names):
            return rec.get("traffic_bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="tile", choices=["tile", "plain", "fused"])
    ap.add_argument("--compare", type=int, default=1,
                    help="also time one step of the other planner modes")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run only the reference copy kernel (counter calibration)")
    ap.add_argument("--workload", default="brick30",
                    choices=["brick30", "batch4096", "grid48", "grid42", "ghz128", "large34", "large36",
                             "ghz33", "ghz36", "targets"],
                    help="brick30 is the headline configuration; the others are the batched, "
                         "decomposition and large-state configurations")
    ap.add_argument("--count", type=int, default=4096, help="batch4096: number of circuits")
    ap.add_argument("--coeffs", type=int, default=27, help="ghz128: log2 of the extracted coefficients")
    ap.add_argument("--cross", type=int, default=12,
                    help="grid42: crossing CZs kept (S of the decomposition, 2^S branches)")
    ap.add_argument("--group", type=int, default=0,
                    help="grid48, ghz128: branches resident at a time (0 = automatic)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="brick30: pick the planner options by timed trials first (then mode auto; "
                         "without it the stored tuning record is used); batch4096: timed-trial "
                         "in-pass fusion width, compared with the cost model")
    ap.add_argument("--tune-out", default=None, help="brick30 --autotune 1: save the tuning table here")
    ap.add_argument("--secondary", type=int, default=1,
                    help="brick30: also run the other configurations once (configs 3-5 and the "
                         "paper's Sec. 3/4 circuits) and attach their lines under \"configs\"")
    ap.add_argument("--block-bits", type=int, default=0,
                    help="large36, ghz36: two-byte block bits B (0 = the library default, 8)")
    ap.add_argument("--tile-fuse", type=int, default=0, help="in-pass fusion width (0 = default)")
    ap.add_argument("--tile-bits", type=int, default=0, help="tile bits (0 = default)")
    ap.add_argument("--low-bits", type=int, default=0, help="contiguous low tile bits (0 = default)")
    ap.add_argument("--pass-gates", type=int, default=0,
                    help="most gates per tile pass (0 = planner's cost model, -1 = no limit)")
    ap.add_argument("--relabel", type=int, default=0,
                    help="tile passes may move qubits onto the low bits (0 = planner's choice, -1 = off)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1912_03243_amd import juqcs
    from paper_1912_03243_amd import workloads as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.copy_calib:
        nbytes = 8 << 30
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        for _ in range(3):
            juqcs.juqcs_copy(dst, src, nbytes, stream)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 launches of {nbytes} bytes")
        return

    if args.workload != "brick30":
        return other_workload(args, juqcs, W, dev, stream)

    n, gates, z = W.workload_brick30()
    zd = torch.from_numpy(z.astype(np.int64)).to(dev)
    outd = torch.empty(2 * z.size, dtype=torch.float64, device=dev)
    log(f"workload: n={n}, {len(gates)} gates, {z.size} bitstrings, mode={args.mode}")

    st = juqcs.State(n, "c128", device=dev, stream=stream)
    explicit = args.tile_bits or args.low_bits or args.tile_fuse or args.pass_gates or args.relabel
    tune, run_mode = (None, args.mode) if explicit else tuned_mode(args, juqcs, st, gates)

    def step(mode, profile):
        st.init(0)
        if mode == "auto":
            o = st.run(gates, mode="auto", profile=profile)
        elif mode == "tile":
            o = st.run(gates, mode=mode, profile=profile, fuse_k=args.tile_fuse,
                       tile_bits=args.tile_bits, low_bits=args.low_bits,
                       pass_gates=args.pass_gates, relabel=args.relabel)
        else:
            o = st.run(gates, mode=mode, profile=profile, fuse_k=FUSE_K_C128)
        st.amplitudes_device(zd, outd)
        nrm = st.norm()
        return o, nrm

    for i in range(args.warmup):
        step(run_mode, True)
        log(f"warmup step {i} done")
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kernel_ms = 0.0
    kbytes = 0.0
    passes = 0
    torch.cuda.synchronize()
    start.record(stream)
    t0 = time.perf_counter()
    mma_flops = 0.0
    marks = []
    for i in range(args.steps):
        o, nrm = step(run_mode, True)
        kernel_ms += o.kernel_ms
        kbytes += o.bytes
        passes += o.passes
        mma_flops += o.mma_flops
        marks.append(torch.cuda.Event(enable_timing=True))
        marks[-1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / args.steps
    per_step = [start.elapsed_time(marks[0])] + [marks[i - 1].elapsed_time(marks[i]) for i in range(1, len(marks))]
    log(f"timed {args.steps} steps: {ms:.2f} ms/step (host wall {1e3 * wall / args.steps:.2f})")

    amps = outd.cpu().numpy()
    amps = amps[0::2] + 1j * amps[1::2]
    check = {"norm_minus_1": nrm - 1.0}
    try:
        # stored FP64 amplitudes of this circuit (written by tests/golden/make_golden.py)
        rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "brick30_amplitudes.txt"),
                          dtype=np.float64, comments="#", ndmin=2)
        gz = rows[:, 0].astype(np.uint64)
        ga = rows[:, 1] + 1j * rows[:, 2]
        assert np.array_equal(gz, z[: gz.size])
        check["oracle_max_abs_err"] = float(np.max(np.abs(amps[: gz.size] - ga)))
        check["oracle_points"] = int(gz.size)
    except OSError as e:
        log(f"no stored oracle amplitudes: {e}")

    ngates = len(gates)
    value = ngates / (ms / 1e3)
    pass_ms = kernel_ms / max(passes, 1)
    achieved = (kbytes / max(passes, 1)) / (pass_ms / 1e3) / 1e9
    per_launch = kbytes / max(passes, 1)
    hbm = {"achieved_GBps": achieved, "peak_GBps": HBM_PEAK_GBPS, "frac": achieved / HBM_PEAK_GBPS,
           "bytes_per_launch": per_launch}
    chosen = tune["mode"] if tune else args.mode
    if chosen == "tile":
        # A tile pass absorbs ~64 gates here: far past the FP64 ridge (about
        # 22 gates per pass), so the pass is bound by arithmetic on chip.
        # achieved = the absorbed gates' algorithmic flops per launch / the
        # average launch time (HIP events on the launch stream).
        flops_launch = gate_flops_per_amp(gates, W) * float(1 << n) * args.steps / max(passes, 1)
        tflops = flops_launch / (pass_ms / 1e3) / 1e12
        roofline = {"bound": "alu", "achieved": tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": tflops / FP64_VECTOR_PEAK_TFLOPS,
                    "traffic": traffic_for(TILE_SOURCES),
                    "kernel": ("k_tile_fixed<double,12,512>" if tune and tune["tile_bits"] == 12
                               else "k_tile_fixed<double,13,1024>"),
                    "flops_per_launch": flops_launch, "avg_launch_ms": pass_ms, "hbm": hbm}
    elif chosen == "fused":
        tf = mma_flops / max(passes, 1) / (pass_ms / 1e3) / 1e12
        roofline = {"bound": "mfma", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "traffic": None, "kernel": "k_fused<F64>",
                    "flops_per_launch": mma_flops / max(passes, 1), "avg_launch_ms": pass_ms, "hbm": hbm}
    else:
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "kernel": chosen,
                    "bytes_per_launch": per_launch, "avg_launch_ms": pass_ms}
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "gate-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": float(np.median(per_step)),
        "ms_per_step_min": float(np.min(per_step)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "brick30: n=30 complex128 state (16 GiB), 20 layers of Haar U(2) "
                               "on every qubit + brick CZ (890 gates, seed 2); init, all gates, "
                               "4096 amplitudes (seed 1002) and the norm per step",
                   "n": n, "gates": ngates, "bitstrings": int(z.size), "mode": chosen,
                   "autotune": tune,
                   "tile_fuse": args.tile_fuse, "tile_bits": args.tile_bits,
                   "pass_gates": args.pass_gates, "relabel": args.relabel,
                   "passes_per_step": passes // args.steps},
        "roofline": roofline,
        "amp_updates_per_s": value * float(1 << n),
        "check": check,
    }

    # in-place stream over the state (every word read and written back in
    # the per-gate passes' access pattern): the practical ceiling of a pass
    nb = st.amps.numel()
    juqcs.juqcs_copy(st.amps, st.amps, nb, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        juqcs.juqcs_copy(st.amps, st.amps, nb, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    stream_gbps = 3 * 2 * nb / (e0.elapsed_time(e1) / 1e3) / 1e9
    result["stream_inplace_GBps"] = stream_gbps
    hbm["frac_of_stream"] = achieved / stream_gbps
    if chosen == "plain":
        result["roofline"]["frac_of_stream"] = achieved / stream_gbps

    if args.compare:
        for mode in ("plain", "fused"):
            if mode == chosen:
                continue
            torch.cuda.synchronize()
            t = time.perf_counter()
            o, _ = step(mode, True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            gbps = o.bytes / (o.kernel_ms / 1e3) / 1e9
            line = {"ms_per_step": el * 1e3, "gate_updates_per_s": ngates / el, "passes": o.passes,
                    "avg_pass_ms": o.kernel_ms / max(o.passes, 1), "achieved_GBps": gbps,
                    "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS,
                                 "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                                 "frac_of_stream": gbps / stream_gbps}}
            if mode == "fused":
                tf = o.mma_flops / (o.kernel_ms / 1e3) / 1e12
                line.update({"mma": "fp64", "fuse_k": FUSE_K_C128,
                             "mfma": {"achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS,
                                      "unit": "TFLOP/s", "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
                                      "flops_per_step": o.mma_flops}})
            result[f"{mode}_step"] = line
            log(f"{mode}: {el * 1e3:.1f} ms for one step, {o.passes} passes")

    st.close()
    del st
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.secondary:
        result["configs"] = secondary_configs(args, juqcs, W, dev, stream)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(n, gates, args.cpu_budget)
    print(json.dumps(result), flush=True)


# The other configurations, each run once after the headline (steps, warmup):
# the 128 GiB complex64 and two-byte states, the 4096-circuit batch (with the
# batch autotuner, the cost model timed beside it), the 48-qubit grid
# decomposition, and the paper's Sec. 3 and Sec. 4 GHZ circuits.
SECONDARY = (("large34", 2, 1), ("large36", 1, 0), ("batch4096", 2, 1), ("grid48", 2, 1),
             ("ghz128", 2, 1), ("ghz33", 2, 1))
SECONDARY_KEYS = ("value", "unit", "ms_per_step", "steps", "warmup", "dtype", "roofline", "check",
                  "amp_updates_per_s", "ms_per_gate", "coefficients_per_s", "cost_model_ms_per_step",
                  "expectations_ms", "tile", "plain", "branch_stats")


def secondary_configs(args, juqcs, W, dev, stream):
    import argparse as _ap
    import torch
    out = {}
    for name, steps, warmup in SECONDARY:
        a = _ap.Namespace(**vars(args))
        a.workload, a.steps, a.warmup = name, steps, warmup
        a.autotune = 1 if name == "batch4096" else 0
        a.tile_fuse = a.tile_bits = a.low_bits = a.pass_gates = a.relabel = 0
        t0 = time.perf_counter()
        try:
            res = other_workload(a, juqcs, W, dev, stream, emit=False)
            line = {k: res[k] for k in SECONDARY_KEYS if k in res}
            line["workload"] = res["config"]["workload"]
            for k in ("passes_per_step", "autotune", "fusion_width_counts", "circuits", "gates", "n"):
                if k in res["config"]:
                    line[k] = res["config"][k]
        except Exception as e:  # a failed configuration is reported, the headline still stands
            line = {"error": f"{type(e).__name__}: {e}"}
        line["wall_s"] = time.perf_counter() - t0
        out[name] = line
        log(f"{name}: {line.get('ms_per_step', line.get('error'))}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def sample_errors(got, want):
    """Errors of sampled amplitudes against the oracle's: relative L2, max
    error over max |phi|, and 1 - fidelity estimated from the samples
    (|<phi|psi>|^2 / (<phi|phi><psi|psi>) over the sampled set)."""
    import numpy as np
    d = got - want
    fid = abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real)
    return {"oracle_points": int(want.size),
            "oracle_rel_l2": float(np.linalg.norm(d) / np.linalg.norm(want)),
            "oracle_max_err_over_max": float(np.abs(d).max() / np.abs(want).max()),
            "oracle_one_minus_fidelity_sampled": float(1.0 - fid)}


def batch_sample_errors(amps, count):
    """The batch's read-out against the stored oracle amplitudes of its
    stratified sample (tests/golden/batch4096s_amplitudes.txt)."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    try:
        from make_golden import load_batch
        ref = load_batch("batch4096s")
    except OSError:
        return {}
    worst_l2 = worst_max = 0.0
    for i, (z, want) in ref.items():
        if i >= count:
            continue
        e = sample_errors(amps[i], want)
        worst_l2 = max(worst_l2, e["oracle_rel_l2"])
        worst_max = max(worst_max, e["oracle_max_err_over_max"])
    return {"oracle_circuits": len(ref), "oracle_worst_rel_l2": worst_l2,
            "oracle_worst_max_err_over_max": worst_max}


def tree_roofline(bst, ms):
    """Roofline of the part-state trees of a decomposition step: the
    algorithmic flops of the gates they simulated over the step time (the
    tile kernel is most of the step, so this is a lower bound on its rate),
    against the FP32 matrix-core peak, with their HBM bytes beside."""
    tf = bst["gate_flops"] / (ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP32_MFMA_PEAK_TFLOPS, "kernel": "k_batch", "flops_per_step": bst["gate_flops"],
            "hbm": {"achieved_GBps": bst["pass_bytes"] / (ms / 1e3) / 1e9,
                    "bytes_per_step": bst["pass_bytes"],
                    "note": "24-qubit part states (128 MiB) are cache-resident: effective"},
            "note": "over the whole step"}


def tuned_mode(args, juqcs, st, gates):
    """Planner options for the tile mode: the stored tuning record's entry
    for this circuit (written by an earlier --autotune 1 run on MI355X), or
    fresh timed trials with --autotune 1 (saved with --tune-out, together
    with the record's other entries).  Returns (entry or None, run mode)."""
    if args.mode != "tile":
        return None, args.mode
    if os.path.exists(TUNING_RECORD):
        juqcs.juqcs_tune_load(TUNING_RECORD)
    if args.autotune:
        os.environ["JUQCS_TUNE_VERBOSE"] = "1"    # one stderr line per timed trial
        t0 = time.perf_counter()
        tune = st.autotune(gates)
        tune["wall_s"] = time.perf_counter() - t0
        tune["source"] = "timed trials in this run"
        if args.tune_out:
            juqcs.juqcs_tune_save(args.tune_out)
    else:
        tune = st.tuned(gates)
        if tune is not None:
            tune["source"] = os.path.relpath(TUNING_RECORD, ROOT)
    log(f"autotune: {tune}")
    return tune, ("auto" if tune is not None else "tile")


def _timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def other_workload(args, juqcs, W, dev, stream, emit=True):
    """Secondary configurations (not the headline line): many small circuits
    in one graph launch, the entangling-gate decomposition, and the
    largest single states in complex64 and two-byte form."""
    import numpy as np
    import torch
    res = {"metric": METRIC, "unit": "gate-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}
    if args.workload == "batch4096":
        t0 = time.perf_counter()
        inst = W.batch_instances(args.count)
        t_gen = time.perf_counter() - t0
        s = torch.cuda.Stream(dev)
        t0 = time.perf_counter()
        b = juqcs.Batch(inst, device=dev, autotune=bool(args.autotune), relabel=args.relabel)
        t_plan = time.perf_counter() - t0
        st = b.stats()
        log(f"batch: {len(inst)} circuits, {st}, generation {t_gen:.1f}s, planning {t_plan:.1f}s")

        def run():
            b.run(s)

        with torch.cuda.stream(s):
            ms = _timed(run, args.steps, args.warmup, s)
            b.wait()
            idx = np.stack([W.batch_bitstrings(i, n) for i, (n, _) in enumerate(inst)])
            amps = b.amplitudes(idx, s)
            norms = b.norms(s)
        cost_model_ms = None
        if args.autotune:
            # the same batch planned by the cost model alone, on the same states
            t0 = time.perf_counter()
            b0 = juqcs.Batch(inst, device=dev, states=b.states, relabel=args.relabel, stream=s)
            t_plan0 = time.perf_counter() - t0
            with torch.cuda.stream(s):
                cost_model_ms = _timed(lambda: b0.run(s), args.steps, args.warmup, s)
                b0.wait()
            b0.close()
            # the autotuned batch wrote the states last for the read-outs above
            log(f"cost-model plan: {cost_model_ms:.1f} ms (planning {t_plan0:.1f}s) vs autotuned {ms:.1f} ms")
        gates = sum(len(g) for _, g in inst)
        amp_updates = sum(len(g) * float(1 << n) for n, g in inst)
        flops = sum(gate_flops_per_amp(g, W) * float(1 << n) for n, g in inst)
        kin = b.fusion()
        check = {"max_abs_norm_minus_1": float(np.max(np.abs(norms - 1.0))),
                 "amplitudes": int(amps.size),
                 "amplitudes_sha256": hashlib.sha256(np.ascontiguousarray(amps).tobytes()).hexdigest()}
        check.update(batch_sample_errors(amps, len(inst)))
        tf = flops / (ms / 1e3) / 1e12
        # algorithmic bytes: the first pass of a circuit writes its state, later passes
        # read and write it (8 bytes per amplitude)
        res.update({
            "value": gates / (ms / 1e3), "ms_per_step": ms, "dtype": "f32",
            "config": {"workload": f"batch{len(inst)}: independent layered circuits, n ~ U{{12..24}}, "
                                   "depth ~ U{10..40} (Haar U(2) + random CZ pairs), complex64, "
                                   "one graph launch (a persistent kernel per pass round)",
                       "circuits": len(inst), "gates": gates, "tile_tasks": st["tasks"],
                       "tile_passes": st["passes"],
                       "fusion_width_counts": {int(k): int((kin == k).sum()) for k in set(kin.tolist())},
                       "autotune": bool(args.autotune), "relabel": args.relabel},
            "amp_updates_per_s": amp_updates / (ms / 1e3),
            "planning_s": t_plan,
            "cost_model_ms_per_step": cost_model_ms,
            # the graph is one persistent tile kernel per pass round: its
            # time is the step; in-tile ops run on FP32 matrix cores and VALU
            "roofline": {"bound": "alu", "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / FP32_MFMA_PEAK_TFLOPS,
                         "kernel": "k_batch", "flops_per_step": flops,
                         "hbm": {"achieved_GBps": 16.0 * st["tasks"] * 8192 / (ms / 1e3) / 1e9,
                                 "note": "tile tasks x 2^13 amplitudes x 16 B; states of n <= 24 "
                                         "are cache-resident, so effective"}},
            "check": check,
        })
        b.close()
    elif args.workload == "grid48":
        circ, side = W.grid_circuit()
        z = W.bitstrings(48, 1024, seed=1005)
        out = {}
        work = juqcs.branch_workspace(48, circ, side, 1, z.size, args.group, True, dev)

        def run():
            out["a"] = juqcs.juqcs_branch_amplitudes(48, circ, side, z, group_size=args.group,
                                                     stream=stream, work=work)

        ms = _timed(run, args.steps, args.warmup, stream)
        bst = juqcs.juqcs_branch_last_stats()
        m = 10
        half_gates = len(circ) - m + 2 * m   # every crossing CZ becomes a diagonal in each half
        res.update({
            "value": (1 << m) * half_gates / (ms / 1e3), "ms_per_step": ms, "dtype": "f32",
            "config": {"workload": "grid48: 6x8 grid, depth 8, Haar U(2) + 4 CZ edge patterns, "
                                   "24|24 cut with m=10 decomposed CZs -> 1024 branch pairs of "
                                   "24-qubit complex64 half-states, each half run as a tree that "
                                   "shares the gates common to its branches; 1024 amplitudes summed "
                                   "over branches in FP64 (value: half-circuit gates of every branch "
                                   "per second, an effective rate since shared gates run once)",
                       "gates": int(len(circ)), "branches": 1 << m, "bitstrings": int(z.size)},
            "roofline": tree_roofline(bst, ms),
            "branch_stats": bst,
            "check": {"sum_abs2_of_1024_amps": float(np.sum(np.abs(out["a"]) ** 2))},
        })
    elif args.workload == "grid42":
        # Section 4's random-circuit runs: 42 qubits cut into two halves of 21,
        # M = 2^20 coefficients; the time per gate grows with 2^S, S the
        # number of decomposed CZs (here the first S crossing CZs are kept)
        rows, cols, depth = 7, 6, 12
        circ, side = W.grid_circuit(rows, cols, depth, seed=7, max_cross=args.cross)
        n = rows * cols
        M = 1 << 20
        z = W.bitstrings(n, M, seed=1007)
        out = {}
        work = juqcs.branch_workspace(n, circ, side, 1, M, args.group, True, dev)

        def run():
            out["a"] = juqcs.juqcs_branch_amplitudes(n, circ, side, z, group_size=args.group,
                                                     stream=stream, work=work)

        ms = _timed(run, args.steps, args.warmup, stream)
        bst = juqcs.juqcs_branch_last_stats()
        a = out["a"]
        S = int(np.sum((side[circ["q0"]] != side[np.maximum(circ["q1"], 0)])
                       & (circ["op"] == W.OP_CZ)))
        res.update({
            "value": len(circ) / (ms / 1e3), "ms_per_step": ms, "dtype": "f32",
            "config": {"workload": f"grid42: 7x6 grid, depth {depth}, Haar U(2) + 4 CZ edge patterns, "
                                   f"21|21 cut with S={S} decomposed CZs -> {1 << S} branch pairs of "
                                   "21-qubit complex64 half-states run as trees; 2^20 coefficients "
                                   "summed over branches in FP64 (value: gates of the 42-qubit circuit "
                                   "per second, the inverse of the paper's time per gate)",
                       "gates": int(len(circ)), "crossings": S, "branches": 1 << S, "bitstrings": M,
                       "group": args.group},
            "ms_per_gate": ms / len(circ),
            "roofline": tree_roofline(bst, ms),
            "branch_stats": bst,
            "check": {"mean_abs2_times_2^n": float(np.mean(np.abs(a) ** 2) * 2.0 ** n)},
        })
    elif args.workload == "ghz128":
        # Section 4's scaling run at its largest size: the GHZ circuit on 128
        # qubits by the Eq. (3) decomposition, M = 2^27 coefficients; the
        # paper reports the elapsed time per gate
        n, nparts = 128, 8
        circ = W.ghz(n)
        side = W.block_parts(n, nparts)
        M = 1 << args.coeffs
        ones = (1 << n) - 1
        z = W.bitstrings_wide(n, M, seed=1006)
        z[:2] = W.ints_to_words([0, ones], n)
        # bitstrings and coefficients resident in HBM for the timed steps
        dz = torch.from_numpy(z.view(np.int64)).to(dev)
        dout = torch.empty(2 * M, dtype=torch.float64, device=dev)
        work = juqcs.branch_workspace(n, circ, side, z.shape[1], M, args.group, False, dev)

        def run():
            juqcs.juqcs_branch_amplitudes_device(n, circ, side, dz, dout, group_size=args.group,
                                                 stream=stream, work=work)

        ms = _timed(run, args.steps, args.warmup, stream)
        bst = juqcs.juqcs_branch_last_stats()
        # the same with host bitstrings in and host coefficients out (PCIe)
        t0 = time.perf_counter()
        host = juqcs.juqcs_branch_amplitudes(n, circ, side, z, group_size=args.group, stream=stream)
        host_ms = (time.perf_counter() - t0) * 1e3
        m = nparts - 1
        a = dout.cpu().numpy().view(np.complex128)
        assert np.array_equal(a, host)
        res.update({
            "value": len(circ) / (ms / 1e3), "ms_per_step": ms, "dtype": "f32",
            "config": {"workload": f"ghz128: GHZ circuit (H(0) + 127 CNOT(i,i+1)) on 128 qubits in "
                                   f"{nparts} parts of 16, the {m} crossing CNOTs decomposed -> "
                                   f"{1 << m} branches of {nparts} complex64 part-states (each part "
                                   "state simulated once per distinct setting of its own crossings); "
                                   f"2^{args.coeffs} coefficients (|0...0>, |1...1> and seeded random "
                                   "strings) summed over all branches in FP64; bitstrings and "
                                   "coefficients resident in HBM (value: gates of the 128-qubit "
                                   "circuit per second, the inverse of the paper's time per gate)",
                       "gates": int(len(circ)), "branches": 1 << m, "bitstrings": M,
                       "group": args.group},
            "ms_per_gate": ms / len(circ),
            "coefficients_per_s": M / (ms / 1e3),
            "host_io_ms": host_ms,
            # the step is dominated by the Eq. (3) sum (FP64 products over
            # the parts for every branch and coefficient)
            "roofline": {"bound": "alu", "achieved": bst["sum_flops"] / (ms / 1e3) / 1e12,
                         "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": bst["sum_flops"] / (ms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                         "kernel": "k_branch_sum_lds" if bst["lds_sum"] else "k_branch_gather_accum",
                         "flops_per_step": bst["sum_flops"],
                         "note": "algorithmic 2^m (6 (P-1) + 2) FP64 flops per coefficient over the "
                                 "whole step (prefix products over the parts skip part of them)"},
            "branch_stats": bst,
            "check": {"amp_all_zero": float(a[0].real), "amp_all_one": float(a[1].real),
                      "nonzero_random": int(np.count_nonzero(a[2:]))},
        })
    elif args.workload == "targets":
        # one per-gate pass per target bit: a dense 2x2 on every bit below the
        # run width and a few above it, c128 at n = 30 and c64 at n = 31 (16
        # GiB each); achieved GB/s = 2 x state bytes / pass time (HIP events)
        u = np.array([[0.6, 0.8j], [0.8j, 0.6]])
        lines = {}
        for dtype, n in (("c128", 30), ("c64", 31)):
            st = juqcs.State(n, dtype, device=dev, stream=stream)
            st.init(0)
            full = 2.0 * (16 if dtype == "c128" else 8) * (1 << n)
            nb = st.amps.numel()
            stream_ms = _timed(lambda: juqcs.juqcs_copy(st.amps, st.amps, nb), max(args.steps, 4), 1, stream)
            per = {"stream": {"ms": stream_ms, "GBps": full / stream_ms / 1e6}}
            for t in list(range(9)) + [n // 2, n - 1]:
                ms = _timed(lambda: st.apply_1q(t, u), max(args.steps, 4), 1, stream)
                per[str(t)] = {"ms": ms, "GBps": full / ms / 1e6, "frac_of_stream": stream_ms / ms}
            lines[f"{dtype} n={n}"] = per
            st.close()
            del st
            torch.cuda.empty_cache()
        worst = min(v["GBps"] for per in lines.values() for k, v in per.items() if k != "stream")
        res.update({
            "value": worst, "unit": "GB/s (slowest target bit)", "ms_per_step": None, "dtype": "f64/f32",
            "config": {"workload": "targets: one dense 2x2 per-gate pass per target bit (0..8, n/2, n-1), "
                                   "c128 n=30 and c64 n=31"},
            "targets": lines,
        })
    elif args.workload in ("ghz33", "ghz36"):
        # the paper's benchmark circuit (Section 3): H on qubit 0, CNOT(i, i+1)
        # for i < n-1, then the expectation values of all qubits; the paper
        # reports the elapsed time per gate
        n, dtype = (33, "c128") if args.workload == "ghz33" else (36, "enc2")
        circ = W.ghz(n)
        st = juqcs.State(n, dtype, device=dev, stream=stream,
                         block_bits=args.block_bits if dtype == "enc2" else 0)
        q = {}
        modes = {}
        tune, tile_mode = tuned_mode(args, juqcs, st, circ)
        for mode in ("tile", "plain"):
            run_as = tile_mode if mode == "tile" else mode

            def run(run_as=run_as):
                st.init(0)
                st.run(circ, mode=run_as)
            steps = args.steps if mode == "tile" else 1
            ms = _timed(run, steps, args.warmup if mode == "tile" else 0, stream)
            st.init(0)
            o = st.run(circ, mode=run_as, profile=True)
            modes[mode] = {"ms_per_circuit": ms, "ms_per_gate": ms / len(circ), "passes": o.passes,
                           "avg_pass_ms": o.kernel_ms / max(o.passes, 1),
                           "achieved_GBps": o.bytes / (o.kernel_ms / 1e3) / 1e9}
            log(f"ghz {mode}: {ms:.1f} ms, {o.passes} passes")

        def expect():
            q["v"] = st.expectations()

        ms_q = _timed(expect, args.steps, args.warmup, stream)
        amps = st.amplitudes(np.array([0, (1 << n) - 1, 1, 1 << (n - 1)], dtype=np.uint64))
        t = modes["tile"]
        res.update({
            "value": len(circ) / ((t["ms_per_circuit"] + ms_q) / 1e3),
            "ms_per_step": t["ms_per_circuit"] + ms_q, "dtype": "f64" if dtype == "c128" else "enc2",
            "config": {"workload": f"{args.workload}: n={n} {dtype} GHZ circuit (H(0) + {n - 1} "
                                   "CNOT(i,i+1)) + expectation values of all qubits; init, gates "
                                   "and expectations per step", "n": n, "gates": len(circ),
                       "autotune": tune},
            "tile": t, "plain": modes["plain"],
            "expectations_ms": ms_q,
            "amp_updates_per_s": len(circ) * float(1 << n) / (t["ms_per_circuit"] / 1e3),
            "check": {"amp0_minus_inv_sqrt2": float(abs(amps[0] - 2 ** -0.5)),
                      "amp_last_minus_inv_sqrt2": float(abs(amps[1] - 2 ** -0.5)),
                      "max_abs_other": float(np.abs(amps[2:]).max()),
                      "max_abs_Q_minus_half": float(np.abs(q["v"] - 0.5).max())},
        })
        st.close()
    else:
        n, dtype = (34, "c64") if args.workload == "large34" else (36, "enc2")
        circ = W.layered_brick(n, 16, seed=3)
        st = juqcs.State(n, dtype, device=dev, stream=stream,
                         block_bits=args.block_bits if dtype == "enc2" else 0)
        info = {}
        explicit = args.tile_bits or args.low_bits or args.tile_fuse or args.pass_gates or args.relabel
        tune, run_mode = (None, "tile") if explicit else tuned_mode(args, juqcs, st, circ)

        def run():
            st.init(0)
            if run_mode == "auto":
                o = st.run(circ, mode="auto", profile=True)
            else:
                o = st.run(circ, mode="tile", profile=True, fuse_k=args.tile_fuse,
                           tile_bits=args.tile_bits, low_bits=args.low_bits,
                           pass_gates=args.pass_gates, relabel=args.relabel)
            info["o"] = (o.passes, o.kernel_ms, o.bytes, o.flops)

        ms = _timed(run, args.steps, args.warmup, stream)
        passes, kms, kb, fl = info["o"]
        nrm = st.norm()
        achieved = kb / (kms / 1e3) / 1e9
        tf = fl / (kms / 1e3) / 1e12
        check = {"norm_minus_1": nrm - 1.0}
        name = "brick34" if args.workload == "large34" else "brick36"
        try:
            rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", f"{name}_amplitudes.txt"),
                              dtype=np.float64, comments="#", ndmin=2)
            want = rows[:, 1] + 1j * rows[:, 2]
            got = st.amplitudes(rows[:, 0].astype(np.uint64))
            check.update(sample_errors(got, want))
        except OSError as e:
            log(f"no stored oracle amplitudes: {e}")
        # norm drift after each layer (outside the timed steps): the circuit
        # again, one layer per run, the FP64 norm read after each
        bounds = [0]
        for layer in range(16):
            bounds.append(bounds[-1] + n + len(range(layer % 2, n - 1, 2)))
        st.init(0)
        drift = []
        for layer in range(16):
            st.run(circ[bounds[layer]:bounds[layer + 1]], mode="tile")
            drift.append(st.norm() - 1.0)
        check["norm_drift_per_layer"] = drift
        res.update({
            "value": len(circ) / (ms / 1e3), "ms_per_step": ms,
            "dtype": "f32" if dtype == "c64" else "enc2",
            "config": {"workload": f"{args.workload}: n={n} {dtype}, 16 brick layers ({len(circ)} gates, "
                                   "seed 3), tile passes", "n": n, "passes_per_step": passes,
                       "relabel": args.relabel, "autotune": tune},
            # passes absorb far more gates than one HBM pass pays for: bound
            # by on-chip arithmetic (FP32 matrix cores for the 8x8 ops, VALU
            # for the rest and for the two-byte codec)
            "roofline": {"bound": "alu", "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / FP32_MFMA_PEAK_TFLOPS,
                         "frac_of_fp32_valu": tf / FP64_VECTOR_PEAK_TFLOPS,
                         "flops_per_launch": fl / passes, "avg_launch_ms": kms / passes,
                         "kernel": (("k_tile_fixed<float,12,512>" if tune and tune["tile_bits"] == 12
                                     else "k_tile_fixed<float,13,1024>") if dtype == "c64"
                                    else "k_tile_enc2_fixed<13>"),
                         "hbm": {"achieved_GBps": achieved, "peak_GBps": HBM_PEAK_GBPS,
                                 "frac": achieved / HBM_PEAK_GBPS, "bytes_per_launch": kb / passes}},
            "amp_updates_per_s": len(circ) * float(1 << n) / (ms / 1e3),
            "check": check,
        })
        st.close()
    if emit:
        print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
