"""Throughput of a large random levelled circuit on one GPU.

    python -m paper_2306_11006_amd.dag [--params large] [--gates 200000]
        [--max-width 65536] [--forms int8 ntt auto] [--seed 1]

The circuit is inputs.random_dag: level widths log-uniform in
[1, max_width] until the gate count is reached, gates NAND/AND/OR/XOR/MUX
reading one wire of the previous level and two earlier ones.  It is
levelised once (cggi_levelize) and, per form, captured as one HIP graph (one
cggi_eval_level per level) and replayed once; the replay is timed.  "auto"
installs the autotuned int8 plan and picks the faster form per level from
the tuned table (paper_2306_11006_amd.tune).
All forms must produce the same wires; the run checks that on every wire
and prints one JSON line per form with bootstraps/s.

Keys and input ciphertexts are uniform random words (seeded): the kernels'
work does not depend on them being valid encryptions.
"""
import argparse
import json
import time

import numpy as np
import torch

from . import cggi, inputs, params, tune
from .circuit import LevelledCircuit


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--params", default="large", choices=list(params.ALL))
    ap.add_argument("--gates", type=int, default=200000)
    ap.add_argument("--max-width", type=int, default=65536)
    ap.add_argument("--forms", nargs="+", default=["int8", "ntt", "auto"],
                    choices=["int8", "ntt", "auto"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tune-max-width", type=int, default=8192)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("dag: no GPU visible (the library runs on HIP "
                         "devices only)")
    p = params.ALL[a.params]
    t0 = time.perf_counter()
    nl = inputs.random_dag(a.seed, a.gates, max_width=a.max_width)
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    print(json.dumps({"circuit": "random_dag", "gates": len(circ.gates),
                      "levels": circ.n_levels,
                      "max_width": int(max(circ.widths)),
                      "bootstraps": circ.bootstraps(),
                      "build_s": round(time.perf_counter() - t0, 2)}),
          flush=True)
    bsk, ksk = inputs.uniform_keys(p, a.seed)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    table = None
    if "auto" in a.forms:
        t1 = time.perf_counter()
        table = tune.load_or_tune(ctx, p, max_width=a.tune_max_width)
        print(json.dumps({"tuned_plan": table["plan"],
                          "tune_s": round(time.perf_counter() - t1, 1)}),
              flush=True)
    wires0 = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    wires0[nl.input_wires] = inputs.uniform_lwe(p, a.seed + 1,
                                                len(nl.input_wires))
    d0 = cggi.to_device(wires0)
    ref = None
    for form in a.forms:
        if form == "auto":
            tune.apply(ctx, table)
        else:
            ctx.int8_plan(None)
        w = d0.clone()
        graph = circ.capture(ctx, form, w, table=table)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        replay = time.perf_counter() - t1
        del graph
        if ref is None:
            ref = w
            same = True
        else:
            same = bool(torch.equal(w, ref))
        ctx.check()
        forms_used = sorted(set(circ.forms_for(form, table)))
        print(json.dumps({
            "form": form, "forms_used": forms_used,
            "graph_replay_s": round(replay, 3),
            "bootstraps_per_s": round(circ.bootstraps() / replay, 1),
            "wires_equal_first_form": same, "params": p.name,
            "data": "uniform random keys and ciphertexts (seeded)"}),
            flush=True)
        if not same:
            raise SystemExit(f"dag: form {form} differs from {a.forms[0]}")
    ctx.close()


if __name__ == "__main__":
    main()
