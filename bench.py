#!/usr/bin/env python3
"""Gate bootstraps per second on one MI355X.

Workload: one level of 1024 independent NAND gates at n=630, N=1024,
Bg=2^7 l=3, key switch base 2^2 t=8 (the default parameter set).  A step is
one cggi_eval_level call over that level: linear pre-op, modulus switch,
accumulator init, 630 CMux steps, sample extraction and key switch for every
gate, writing the 1024 output wires.  Inputs and keys are resident in HBM
before timing starts.  The int8-MFMA form gives `value`; the NTT form is
timed on the same batch and reported beside it.  Each form's step is also
captured once as a HIP graph and replayed `steps` times (`graph_replay`:
mean and median per replay, and whether the replays reproduce the eager
outputs).

Beside the main line: the mixed level of 16,384 independent gates with
opcodes uniform over NAND/AND/OR/XOR/MUX (19,727 bootstraps, MUX counting
two) timed for both forms (`mixed_level_16384`), the level chain of a
one-gate and a 64-gate level (`level_chain`: graph replay per level
against the summed bootstrap and key-switch kernel time), and a one-gate
level in latency mode (`narrow_level`).

Keys and ciphertexts are seeded uniform arrays: real ones are
indistinguishable from uniform under the LWE assumption and every kernel's
work is independent of the values.  Every output row of the 1024-NAND and
16,384-gate levels is compared with the oracle's through the per-row
digests the oracle wrote (tests/golden/digests.py); the CPU baseline runs
the plain C oracle on a bounded sample of the same gates (and checks those
gates' GPU outputs bit for bit).

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("gate bootstraps/sec on 1 MI355X (N=1024), int8-MFMA vs NTT form, "
          "bit-exact")
PEAK_INT8_TOPS = 5000.0      # dense int8 MFMA, MI355X
DIGESTS = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_sha256(path):
    """sha256 of a C++/HIP source with // comments and blank lines removed
    (a comment edit does not change the kernel the counters describe)."""
    import hashlib
    lines = []
    for line in open(path, encoding="utf-8"):
        code = line.split("//", 1)[0].strip()
        if code:
            lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def stored_traffic(profile="profiles/eval_level_1024_nand_default.md",
                   kernel=None):
    """HBM bytes per launch of the int8 bootstrap kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs (each scaled by the factor the same
    counter showed for a copy of known size), or None when the counters were
    taken on another version of the kernel source or (when `kernel` is
    given) on another kernel."""
    try:
        text = open(os.path.join(ROOT, profile)).read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        if line.startswith("traffic-") and ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kernel is not None and kv["traffic-kernel"] != kernel:
            return None
        if code_sha256(os.path.join(ROOT, kv["traffic-source"])) != \
                kv["traffic-code-sha256"]:
            return None
        kib = (float(kv["traffic-fetch-kib"]) * float(kv["traffic-fetch-factor"])
               + float(kv["traffic-write-kib"]) *
               float(kv["traffic-write-factor"]))
    except (KeyError, ValueError, OSError):
        return None
    return int(round(kib * 1024))


def int8_ops_per_bootstrap(p, kind="tiles4"):
    """int8 MFMA operations one bootstrap issues: the block-Toeplitz GEMM of
    every CMux step, 2 * 2N * (2lN * S) * 4 limbs * n; the Karatsuba kernel
    (kind kara2) computes each length-N negacyclic product as three of
    length N/2, so it issues 3/4 of that."""
    S = 1 if p.bg_bit <= 7 else 2
    full = 2 * (2 * p.N) * (2 * p.l * p.N * S) * 4 * p.n
    return full * 3 // 4 if kind == "kara2" else full


def int8_kind_for(plan, bootstraps):
    """Kernel kind of an int8 plan [(kind, cap)] that takes a batch."""
    for kind, cap in plan:
        if bootstraps <= cap:
            return kind
    return plan[-1][0]


def int8_kernel_name(p, kind):
    L, S = (p.l, 1) if p.bg_bit <= 7 else (p.l, 2)
    if (L, S) not in ((3, 1), (2, 2)):
        L, S = 0, 0
    if kind == "kara2":
        # the Karatsuba kernel fixes the digit width for l = 3, Bg = 2^7
        bb = 7 if (L, S) == (3, 1) and p.bg_bit == 7 else 0
        return f"k_bootstrap_int8_kara<{p.N}, {L}, {S}, {bb}>"
    tiles = {"tiles1": 1, "tiles2": 2, "tiles4": 4}.get(kind, 4)
    return f"k_bootstrap_int8<{p.N}, {L}, {S}, {tiles}>"


def ntt_mulmods_per_bootstrap(p):
    logN = p.N.bit_length() - 1
    per_ntt = (p.N // 2) * logN
    return p.n * ((2 * p.l + 2) * per_ntt + 2 * p.l * 2 * p.N)


def bootstraps_of(gates_np):
    """Bootstraps of a gate list: MUX two, NOT/COPY/CONST none, others one."""
    from paper_2306_11006_amd import inputs
    return int(sum(inputs.BOOTSTRAPS[int(o)] for o in gates_np[:, 0]))


def digest_mismatches(name, rows):
    """Row indices whose SHA-256 prefix differs from the oracle's stored
    digest of case `name` (tests/golden/<name>.digests), or None when no
    digest file exists."""
    import hashlib
    import numpy as np
    path = os.path.join(DIGESTS, name + ".digests")
    if not os.path.exists(path):
        return None
    want = [ln.strip() for ln in open(path)
            if ln.strip() and not ln.startswith("#")]
    a = np.ascontiguousarray(rows, dtype="<u4")
    if len(a) != len(want):
        return list(range(len(a)))
    return [i for i, r in enumerate(a)
            if hashlib.sha256(r.tobytes()).hexdigest()[:len(want[i])] !=
            want[i]]


def host_cpu():
    """(logical CPUs, CPUs this process may run on, CPU model name)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return os.cpu_count() or 1, aff, model


def cpu_baseline(p, bsk, ksk, wires_np, gates_np, out_gpu, min_gates,
                 min_seconds, threads):
    """Time the oracle on the first gates of the batch with `threads` host
    threads, one round of `threads` gates at a time, until at least
    `min_gates` gates and `min_seconds` of wall time are done (or the batch
    is exhausted); compare those gates' outputs with the GPU's."""
    import numpy as np
    import oracle as O
    O.lib()

    def one(g):
        op, a, b, _, _ = gates_np[g]
        return O.gate(p, int(op), bsk, ksk, wires_np[a], wires_np[b])

    G = len(gates_np)
    outs = []
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        while len(outs) < G:
            done = len(outs)
            if done >= min_gates and time.perf_counter() - t0 >= min_seconds:
                break
            idx = range(done, min(G, done + threads))
            outs.extend(ex.map(one, idx))
    wall = time.perf_counter() - t0
    # out_gpu holds the output wires in gate order
    ok = all(np.array_equal(o, out_gpu[g]) for g, o in enumerate(outs))
    return len(outs) / wall, len(outs), wall, ok


def time_level(ctx, form, gates, wires, steps, warmup, out_rows,
               bootstraps):
    """Eager steps of one cggi_eval_level (HIP events around the timed
    region, the library's kernel events inside it), then the same level
    captured once as a HIP graph and replayed `steps` times.  Returns the
    figures and the output rows of the eager run."""
    import numpy as np
    import torch
    from paper_2306_11006_amd import cggi
    G = gates.shape[0]
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.eval_level(form, gates, wires)
    torch.cuda.synchronize()
    ctx.profile(True)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        ctx.eval_level(form, gates, wires)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    bs_ms, bs_n, ks_ms, ks_n = ctx.profile_read()
    ctx.profile(False)
    ctx.check()        # a latency-mode time-out would void the figures
    out = cggi.to_host(wires[out_rows])
    r = dict(ms_per_step=ms, bs_kernel_ms=bs_ms / max(bs_n, 1),
             ks_kernel_ms=ks_ms / max(ks_n, 1),
             bootstraps_per_s=bootstraps * 1000.0 / ms,
             gates_per_s=G * 1000.0 / ms)
    # the same step captured once as a HIP graph: one warm-up replay, then
    # `steps` replays, each bracketed by events on the replay stream
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        ctx.eval_level(form, gates, wires)
    graph.replay()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for k in range(steps):
        graph.replay()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(steps))
    gms = evs[0].elapsed_time(evs[-1]) / steps
    ctx.check()
    same = np.array_equal(cggi.to_host(wires[out_rows]), out)
    del graph
    r["graph"] = dict(replays=steps, ms_per_step=round(gms, 4),
                      median_ms=round(per[len(per) // 2], 4),
                      bootstraps_per_s=round(bootstraps * 1000.0 / gms, 1),
                      outputs_equal_eager=bool(same))
    return r, out


def level_chain(ctx, p, dev, widths=(1, 64), reps=20):
    """Per level of `w` NAND gates (int8 form): graph replay ms per level
    against the bootstrap and key-switch kernel ms the library's events
    measure eagerly; the difference is the rest of the level's launch
    chain (slot map, pre-op) and the gaps between its kernels."""
    import numpy as np
    import torch
    from paper_2306_11006_amd import cggi, inputs
    out = {}
    for w in widths:
        idx = np.arange(w, dtype=np.int32)
        z = np.zeros(w, np.int32)
        g = cggi.to_device(np.stack([z, 2 * idx, 2 * idx + 1, z, 2 * w + idx],
                                    axis=1).astype(np.int32), dev)
        wires = cggi.to_device(inputs.uniform_lwe(p, 900 + w, 3 * w), dev)
        ctx.reserve(w)
        ctx.eval_level("int8", g, wires)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.eval_level("int8", g, wires)
        bm, bn, km, kn = ctx.profile_read()
        ctx.profile(False)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            for _ in range(reps):
                ctx.eval_level("int8", g, wires)
        graph.replay()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ctx.check()
        del graph
        gms = e0.elapsed_time(e1) / reps
        kms = (bm + km) / reps
        out[str(w)] = dict(graph_ms_per_level=round(gms, 4),
                           kernel_ms_per_level=round(kms, 4),
                           chain_overhead_frac=round(1.0 - kms / gms, 4))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--gates", type=int, default=1024)
    ap.add_argument("--forms", default="int8,ntt")
    ap.add_argument("--cpu-sample", type=int, default=16,
                    help="least gates the oracle runs for the CPU baseline "
                         "(0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="least wall time of the CPU baseline sample")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="timed steps of the 16,384-gate mixed level (0: "
                         "skip)")
    ap.add_argument("--seed", type=int, default=2306)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first "
                         "(reference kernel for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the batched bootstrap runs on "
              "a single MI355X (multi-GPU sharding of a level is a design "
              "note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2306_11006_amd import cggi, inputs, params

    p = params.DEFAULT
    G = args.gates
    forms = [f for f in args.forms.split(",") if f]
    log(f"[bench] params n={p.n} N={p.N} Bg=2^{p.bg_bit} l={p.l} "
        f"KS 2^{p.ks_base_bit}x{p.ks_t}; {G} NAND gates; forms {forms}")
    bsk, ksk = inputs.uniform_keys(p, args.seed)
    wires_np = inputs.uniform_lwe(p, args.seed + 1, 3 * G)
    idx = np.arange(G, dtype=np.int32)
    gates_np = np.stack([np.zeros(G, np.int32), 2 * idx, 2 * idx + 1,
                         np.zeros(G, np.int32), 2 * G + idx], axis=1)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = cggi.Context(p, cggi.to_device(bsk, dev), cggi.to_device(ksk, dev),
                       forms=forms)
    ctx.reserve(G)
    gates = cggi.to_device(gates_np.astype(np.int32), dev)
    wires = cggi.to_device(wires_np, dev)
    stream = torch.cuda.current_stream()
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        a = torch.empty(nel, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    res = {}
    outs = {}
    for form in forms:
        res[form], outs[form] = time_level(ctx, form, gates, wires,
                                           args.steps, args.warmup,
                                           out_rows=slice(2 * G, 3 * G),
                                           bootstraps=G)
        r0 = res[form]
        log(f"[bench] form={form}: {r0['ms_per_step']:.3f} ms/step, "
            f"bootstrap kernel {r0['bs_kernel_ms']:.3f} ms, key switch "
            f"{r0['ks_kernel_ms']:.3f} ms")
    forms_agree = (len(outs) < 2 or
                   all(np.array_equal(outs[forms[0]], outs[f]) for f in forms))

    main_form = "int8" if "int8" in res else forms[0]
    r = res[main_form]
    # every output row against the oracle's digests (the benchmark's own
    # seeds only: other seeds have no stored digests)
    oracle_rows = {}
    if args.seed == 2306 and G == 1024:
        for f in forms:
            bad = digest_mismatches("level1024_nand_uniform", outs[f])
            oracle_rows[f] = None if bad is None else len(outs[f]) - len(bad)
    mm_ceiling = None
    if "ntt" in res:
        mm_ceiling = cggi.measure_mulmod(20000)
        log(f"[bench] bare Goldilocks multiply-mod loop: {mm_ceiling:.3f} "
            "T/s")

    def ntt_roof(rn, bootstraps):
        mm = ntt_mulmods_per_bootstrap(p) * bootstraps
        ach = mm / (rn["bs_kernel_ms"] * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(ach, 3),
                "peak": round(mm_ceiling, 3), "unit": "Tmulmod/s",
                "frac": round(ach / mm_ceiling, 4),
                "peak_how": "measured: bare loop of the NTT form's Goldilocks "
                            "multiply-mod, NTT launch shape "
                            "(cggi_measure_mulmod)",
                "kernel": "k_bootstrap_ntt<1024, 512>",
                "per_launch": f"{bootstraps} bootstraps x "
                              f"{ntt_mulmods_per_bootstrap(p):.4g} "
                              "multiply-mods"}

    plan = ctx.int8_plan_get() if "int8" in res else []

    def int8_roof(rr, bootstraps):
        kind = int8_kind_for(plan, bootstraps)
        ops = int8_ops_per_bootstrap(p, kind)
        ach = ops * bootstraps / (rr["bs_kernel_ms"] * 1e-3) / 1e12
        r = {"bound": "mfma", "achieved": round(ach, 1),
             "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
             "frac": round(ach / PEAK_INT8_TOPS, 4),
             "kernel": int8_kernel_name(p, kind),
             "per_launch": f"{bootstraps} bootstraps x {ops:.4g} int8 ops"}
        if kind == "kara2":
            # the same bootstraps priced at the full-length Toeplitz GEMM
            full = int8_ops_per_bootstrap(p)
            r["schoolbook_equivalent_tops"] = round(
                full * bootstraps / (rr["bs_kernel_ms"] * 1e-3) / 1e12, 1)
        return r

    if main_form == "int8":
        roof = int8_roof(r, G)
        roof.update({
            "traffic": (stored_traffic(kernel=roof["kernel"]) if G == 1024
                        else None),
            "traffic_unit": "HBM bytes per launch (rocprofv3 counters)"})
    else:
        roof = ntt_roof(r, G)
        roof["traffic"] = None

    if main_form == "int8" and roof.get("traffic"):
        # the HBM side of the same launch: measured bytes over its duration
        gbs = roof["traffic"] / (r["bs_kernel_ms"] * 1e-3) / 1e9
        roof["traffic_gb_per_s"] = round(gbs, 1)
        roof["traffic_frac_of_hbm"] = round(gbs / 8000.0, 5)
    if main_form == "int8":
        # what the GPU sustains for this MFMA with random vs zero operand
        # bits (power limit); the published peak assumes the top clock
        ceil_rand = cggi.measure_int8_mfma(40000, True)
        ceil_zero = cggi.measure_int8_mfma(40000, False)
        log(f"[bench] bare int8 MFMA loop: {ceil_rand:.0f} TOP/s random "
            f"operands, {ceil_zero:.0f} TOP/s zero operands")
        roof["measured_ceiling"] = {
            "random_operands": round(ceil_rand, 1),
            "zero_operands": round(ceil_zero, 1), "unit": "TOP/s",
            "frac_of_random": round(roof["achieved"] / ceil_rand, 4),
            "how": "bare v_mfma_i32_32x32x32_i8 loop, one 8-wave workgroup "
                   "per CU (cggi_measure_int8_mfma)"}

    line = {
        "metric": METRIC, "value": round(r["bootstraps_per_s"], 1),
        "unit": "bootstraps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8" if main_form == "int8" else "u64",
        "data": "synthetic",
        "config": {"workload": f"one level of {G} independent NAND gates, "
                               "n=630 N=1024 Bg=2^7 l=3 KS base 2^2 t=8",
                   "form": main_form, "batch": G, "gates_per_step": G,
                   "bootstraps_per_step": G},
        "roofline": roof,
        "graph_replay": res[main_form]["graph"],
    }
    if "ntt" in res and main_form != "ntt":
        rn = res["ntt"]
        line["ntt_form"] = {
            "value": round(rn["bootstraps_per_s"], 1),
            "ms_per_step": round(rn["ms_per_step"], 4),
            "graph_replay": rn["graph"],
            "roofline": ntt_roof(rn, G)}
        line["int8_over_ntt"] = round(r["bootstraps_per_s"] /
                                      rn["bootstraps_per_s"], 3)
    line["forms_bit_identical"] = bool(forms_agree)
    if oracle_rows:
        line["outputs_equal_oracle"] = {
            f: (None if v is None else f"{v}/{G} rows")
            for f, v in oracle_rows.items()}
    line["kernel_ms"] = {f: {"bootstrap": round(v["bs_kernel_ms"], 4),
                             "keyswitch": round(v["ks_kernel_ms"], 4)}
                         for f, v in res.items()}

    if args.mixed_steps > 0:
        # the 16,384-gate mixed level (opcodes uniform over NAND, AND, OR,
        # XOR, MUX; seeds of the oracle's stored digests)
        MG = 16384
        mbsk, mksk = inputs.uniform_keys(p, 77)
        mgates_np = inputs.random_gate_batch(78, MG)
        mwires_np = np.zeros((4 * MG, p.n + 1), dtype=np.uint32)
        mwires_np[: 3 * MG] = inputs.uniform_lwe(p, 79, 3 * MG)
        MB = bootstraps_of(mgates_np)
        mctx = cggi.Context(p, cggi.to_device(mbsk, dev),
                            cggi.to_device(mksk, dev), forms=forms)
        mctx.reserve(MG)
        mg = cggi.to_device(mgates_np, dev)
        mw = cggi.to_device(mwires_np, dev)
        mixed = {"workload": f"one level of {MG} independent gates, opcodes "
                             "uniform over NAND/AND/OR/XOR/MUX, n=630 N=1024",
                 "gates": MG, "bootstraps": MB, "steps": args.mixed_steps}
        mouts = {}
        for f in forms:
            log(f"[bench] mixed level form={f}: {args.mixed_steps} steps")
            mr, mouts[f] = time_level(mctx, f, mg, mw, args.mixed_steps, 1,
                                      out_rows=slice(3 * MG, 4 * MG),
                                      bootstraps=MB)
            bad = digest_mismatches("mixed16384_uniform", mouts[f])
            mixed[f] = {
                "bootstraps_per_s": round(mr["bootstraps_per_s"], 1),
                "gates_per_s": round(mr["gates_per_s"], 1),
                "ms_per_step": round(mr["ms_per_step"], 3),
                "kernel_ms": {"bootstrap": round(mr["bs_kernel_ms"], 3),
                              "keyswitch": round(mr["ks_kernel_ms"], 3)},
                "graph_replay": mr["graph"],
                "roofline": (int8_roof(mr, MB) if f == "int8"
                             else ntt_roof(mr, MB)),
                "outputs_equal_oracle": (None if bad is None else
                                         f"{MG - len(bad)}/{MG} rows")}
        if len(mouts) == 2:
            mixed["forms_bit_identical"] = bool(
                np.array_equal(mouts["int8"], mouts["ntt"]))
        line["mixed_level_16384"] = mixed
        mctx.close()
        del mg, mw

    if "int8" in res:
        line["level_chain"] = level_chain(ctx, p, dev)
    if "int8" in res and ctx.latency_groups() > 0:
        # a narrow level: one NAND gate's bootstrap in latency mode (eight
        # workgroups on eight CUs) and on the one-workgroup kernel
        one = wires[:1].clone()
        big = torch.empty((1, p.N + 1), dtype=torch.int32, device=dev)
        narrow = {}
        for mode, on in (("latency_mode_ms", True), ("one_workgroup_ms",
                                                      False)):
            ctx.latency_mode(on)
            ctx.bootstrap("int8", one, big)
            torch.cuda.synchronize()
            ctx.profile(True)
            for _ in range(3):
                ctx.bootstrap("int8", one, big)
            bms, bn, _, _ = ctx.profile_read()
            ctx.profile(False)
            narrow[mode] = round(bms / max(bn, 1), 3)
        ctx.latency_mode(True)
        try:
            ctx.check()
            line["narrow_level"] = dict(
                bootstraps=1, **narrow,
                kernels=["k_bootstrap_int8_split<1024, 3, 1, 8>",
                         "k_bootstrap_int8<1024, 3, 1, 1>"])
        except cggi.CggiError as e:
            # a latency-mode wait timed out (e.g. CUs taken by another
            # process): the figures above are void, the main line stands
            line["narrow_level"] = {"error": str(e)}

    if args.cpu_sample > 0:
        nproc, aff, model = host_cpu()
        # the GPU machine gives one GPU's job a share of 16 host threads
        # (OMP_NUM_THREADS there), whatever the machine's core count
        share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or aff
        threads = max(1, min(share, aff))
        log(f"[bench] cpu baseline: oracle, {threads} threads ({nproc} "
            f"logical CPUs, {aff} usable, {model}), at least "
            f"{args.cpu_sample} gates and {args.cpu_seconds:g} s")
        rate, sample, wall, ok = cpu_baseline(
            p, bsk, ksk, wires_np, gates_np, outs[main_form],
            args.cpu_sample, args.cpu_seconds, threads)
        line["cpu_baseline"] = {
            "value": round(rate, 3), "unit": "bootstraps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {sample} of the {G} NAND gates (pre-op, "
                      f"bootstrap, key switch each), {wall:.1f} s wall",
            "gpu_outputs_match": bool(ok),
            "host": {"logical_cpus": nproc, "usable_cpus": aff,
                     "cpu_model": model,
                     "threads_used": threads}}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
