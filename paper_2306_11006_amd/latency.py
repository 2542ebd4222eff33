"""End-to-end latency of encrypted integer arithmetic on one GPU.

    python -m paper_2306_11006_amd.latency [--op add mul uneven] [--bits 32]
        [--form int8 ntt] [--reps 5] [--params default]

For every (operation, circuit design, form) it builds the netlist
(paper_2306_11006_amd.arith), levelises it once, and times the whole circuit
(one cggi_eval_level call per level, ArctyrEX Section 4.2) from the first
level's launch to the last level's completion, with the input ciphertexts
already in device memory; it also times the same run bracketed by the
upload of the input ciphertexts from pinned host memory and the download of
the output ciphertexts (the transfer-inclusive latency), and a replay of the
whole circuit captured as one HIP graph.  One JSON line per case.

Every figure is guarded: after each case the context's latency-mode error
word is checked (a timed-out latency-mode launch exits early and would time
as almost nothing), and when both forms run, the int8 form's final wires
must equal the NTT form's on every coefficient.  A failed check exits with
a non-zero status after printing what failed.

Keys and input ciphertexts are uniform random words of the right shapes
(seeded): the kernels' work and timing do not depend on whether the words
form a valid encryption, and no decryption is made here.
"""
import argparse
import json
import statistics
import time

import numpy as np
import torch

from . import arith, cggi, inputs, params
from .circuit import LevelledCircuit

STYLES = {"add": ("ripple", "prefix"), "mul": ("array", "tree"),
          "uneven": ("ripple+array",)}


def build(op, bits, style):
    """(netlist, input wires, output wires) of one circuit.  "uneven" is the
    uneven-level workload: a bits-wide ripple-carry adder beside a bits x
    bits array multiplier (inputs.adder_multiplier_circuit)."""
    if op == "add":
        nl, io = arith.adder(bits, style)
        return nl, list(io["a"]) + list(io["b"]), list(io["sum"])
    if op == "mul":
        nl, io = arith.multiplier(bits, style)
        return nl, list(io["a"]) + list(io["b"]), list(io["prod"])
    nl, io = inputs.adder_multiplier_circuit(bits)
    return (nl, list(io["a"]) + list(io["b"]) + list(io["x"]) +
            list(io["y"]), list(io["sum"]) + list(io["prod"]))


def time_case(ctx, p, form, nl, ins, outs, reps, seed):
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    ctx.reserve(max(circ.widths))
    host_in = torch.from_numpy(
        inputs.uniform_lwe(p, seed, len(ins)).view(np.int32)).pin_memory()
    host_out = torch.empty((len(outs), p.n + 1), dtype=torch.int32,
                           pin_memory=True)
    d_ins = torch.tensor(ins, dtype=torch.int64, device="cuda")
    d_outs = torch.tensor(outs, dtype=torch.int64, device="cuda")
    wires = torch.zeros((nl.n_wires, p.n + 1), dtype=torch.int32,
                        device="cuda")
    wires[d_ins] = host_in.to("cuda")

    def resident():
        circ.run(ctx, form, wires)

    def with_transfers():
        wires.index_copy_(0, d_ins, host_in.to("cuda", non_blocking=True))
        circ.run(ctx, form, wires)
        host_out.copy_(wires.index_select(0, d_outs), non_blocking=True)

    def timed(fn):
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t0) * 1e3)
        return out

    resident()                        # warm-up (also loads the kernels)
    torch.cuda.synchronize()
    eager = timed(resident)
    moved = timed(with_transfers)
    graph = circ.capture(ctx, form, wires)
    graph.replay()
    torch.cuda.synchronize()
    replay = timed(graph.replay)
    del graph
    ctx.check()        # raises CggiError E_TIMEOUT after a latency time-out
    return circ, eager, moved, replay, wires.cpu()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--op", nargs="+", default=["add", "mul"],
                    choices=["add", "mul", "uneven"])
    ap.add_argument("--style", nargs="+", default=None,
                    help="circuit designs (default: all of the operation's)")
    ap.add_argument("--bits", type=int, default=32)
    ap.add_argument("--form", nargs="+", default=["int8", "ntt"],
                    choices=list(cggi.FORMS))
    ap.add_argument("--params", default="default", choices=list(params.ALL))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("latency: no GPU visible (the library runs on HIP "
                         "devices only)")
    p = params.ALL[a.params]
    bsk, ksk = inputs.uniform_keys(p, a.seed)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk),
                       forms=tuple(a.form))
    failed = False
    for op in a.op:
        for style in a.style or STYLES[op]:
            if style not in STYLES[op]:
                continue
            nl, ins, outs = build(op, a.bits, style)
            final = {}
            for form in a.form:
                try:
                    circ, eager, moved, replay, final[form] = time_case(
                        ctx, p, form, nl, ins, outs, a.reps, a.seed + 1)
                except cggi.CggiError as e:
                    print(json.dumps({"circuit": f"{op}{a.bits}-{style}",
                                      "form": form, "error": str(e)}),
                          flush=True)
                    failed = True
                    continue
                agree = None
                if len(final) == 2:
                    agree = bool(torch.equal(final["int8"], final["ntt"]))
                    failed |= not agree
                print(json.dumps({
                    "circuit": f"{op}{a.bits}-{style}", "form": form,
                    "params": p.name, "gates": int(len(circ.gates)),
                    "bootstraps": circ.bootstraps(),
                    "levels": circ.n_levels,
                    "max_width": int(max(circ.widths)),
                    "latency_ms": round(statistics.median(eager), 2),
                    "latency_ms_min": round(min(eager), 2),
                    "transfer_inclusive_ms": round(statistics.median(moved),
                                                   2),
                    "graph_replay_ms": round(statistics.median(replay), 2),
                    "ms_per_level": round(statistics.median(eager) /
                                          circ.n_levels, 3),
                    "reps": a.reps, "checked": "ctx.check ok",
                    "forms_agree": agree,
                    "data": "uniform random keys and "
                    "ciphertexts (seeded)"}), flush=True)
    ctx.close()
    if failed:
        raise SystemExit("latency: a check failed (see the lines above)")


if __name__ == "__main__":
    main()
