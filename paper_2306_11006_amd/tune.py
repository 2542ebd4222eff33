"""Autotuner of the int8 form's kernel plan (and of the form per level width).

The int8 form has seven kernels for a batch of bootstraps (cggi.KINDS):
latency mode with eight, four or two workgroups per column tile, one
workgroup per 1, 2 or 4 column tiles, and the Karatsuba kernel (three
half-length products per negacyclic product).  All give bit-identical results; which is
fastest depends on the batch width, the parameter set and the GPU.  The
tuner times every kernel that can take each width of a grid (one
cggi_bootstrap_batch per measurement under a plan that forces the kernel,
HIP events around the launch), keeps the fastest per width, and compresses
the winners into a plan of (kind, cap) entries: entry k takes the batches
of cap[k-1] + 1 .. cap[k] bootstraps, so a width between two grid points
goes to the kernel that won the larger one.  It also times the NTT form per
width, so a caller can pick the faster form per level (best_form; at
N = 2048 the NTT form wins).

Tables are cached as JSON keyed by parameter set, device, CU count and the
library build (cache directory: $CGGI_TUNE_CACHE, else ~/.cache/cggi_tune).

    python -m paper_2306_11006_amd.tune [--params default] [--max-width 4096]

Input ciphertexts and keys are uniform random words (seeded): the kernels'
work does not depend on them being valid encryptions.
"""
import argparse
import bisect
import hashlib
import json
import os

import torch

from . import cggi, inputs, params

MAX_CAP = cggi.INT32_MAX


def widths_grid(limits, cus, gpt, max_width=4096):
    """Batch widths to time: powers of two, the latency-mode limits and the
    one-, two- and four-tiles-per-CU boundaries (each with its successor),
    up to max_width."""
    pts = {1 << k for k in range(max_width.bit_length()) if 1 << k <= max_width}
    for b in (limits.get("split8", 0), limits.get("split4", 0),
              limits.get("split2", 0), cus * gpt,
              2 * cus * gpt, 4 * cus * gpt):
        for w in (b, b + 1):
            if 1 <= w <= max_width:
                pts.add(int(w))
    pts.add(max_width)
    return sorted(pts)


MAX_ENTRIES = 8          # cggi_ctx_int8_plan takes at most eight entries


def plan_from_winners(winners, max_entries=MAX_ENTRIES):
    """[(width, kind)] sorted by width -> plan [(kind, cap)]: runs of one
    kind merge into one entry capped at the run's last width; the last entry
    holds every larger batch.  While there are more than `max_entries`
    entries, the run with the fewest winning widths (the first such, never
    the catch-all last entry) is merged into the run after it, which then
    also takes the smaller widths; that keeps every latency-mode cap within
    its kind's limit, since a run's cap never grows."""
    runs = []                                   # [kind, [widths]]
    for w, k in winners:
        if runs and runs[-1][0] == k:
            runs[-1][1].append(w)
        else:
            runs.append([k, [w]])
    if not runs:
        return [("tiles4", MAX_CAP)]
    if runs[-1][0].startswith("split"):
        runs.append(["tiles4", []])
    while len(runs) > max_entries:
        i = min(range(len(runs) - 1), key=lambda j: len(runs[j][1]))
        runs[i + 1][1][:0] = runs[i][1]
        del runs[i]
        merged = []
        for k, ws in runs:
            if merged and merged[-1][0] == k:
                merged[-1][1].extend(ws)
            else:
                merged.append([k, ws])
        runs = merged
    plan = [(k, ws[-1]) for k, ws in runs[:-1]]
    plan.append((runs[-1][0], MAX_CAP))
    return plan


def best_form(table, bootstraps):
    """'int8' or 'ntt', whichever the table timed faster at the smallest grid
    width holding `bootstraps` (the largest width beyond the grid)."""
    forms = table.get("forms")
    if not forms:
        return "int8"
    ws = sorted(int(w) for w in forms)
    i = min(bisect.bisect_left(ws, int(bootstraps)), len(ws) - 1)
    t = forms[str(ws[i])]
    if "ntt" in t and t["ntt"] < t["int8"]:
        return "ntt"
    return "int8"


def cache_key(p, device_name, cus):
    with open(cggi.LIB_PATH, "rb") as f:
        build = hashlib.sha256(f.read()).hexdigest()[:12]
    dev = "".join(ch if ch.isalnum() else "-" for ch in device_name)
    return (f"{p.name}-n{p.n}-N{p.N}-bg{p.bg_bit}-l{p.l}-ks{p.ks_base_bit}x"
            f"{p.ks_t}-{dev}-{cus}cu-{build}")


def cache_dir():
    return os.environ.get("CGGI_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "cggi_tune"))


def _force(ctx, kind, limits):
    """Plan that sends every batch within the kind's limit to `kind`."""
    if kind.startswith("split"):
        ctx.int8_plan([(kind, limits[kind]), ("tiles4", MAX_CAP)])
    else:
        ctx.int8_plan([(kind, MAX_CAP)])


def _time(ctx, form, x, out, reps):
    """Mean kernel ms of `reps` bootstraps of x into out.  The context's
    latency-mode error word is checked afterwards: a timed-out latency-mode
    launch exits early and would otherwise time as almost nothing (raises
    CggiError E_TIMEOUT)."""
    ctx.bootstrap(form, x, out)          # warm-up
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        ctx.bootstrap(form, x, out)
    ms, n, _, _ = ctx.profile_read()
    ctx.profile(False)
    ctx.check()
    return ms / max(n, 1)


def autotune(ctx, p, widths=None, reps=3, time_ntt=True, seed=1,
             max_width=4096):
    """Time every int8 kernel (and the NTT form) per width; return the table
    {"plan": [(kind, cap)], "times": {w: {kind: ms}}, "forms": {w: {form:
    ms}}, ...}.  Every timed kernel's outputs must equal those of the first
    one timed at that width (the NTT form when the context has it), else
    RuntimeError.  The context's plan is restored to the built-in one."""
    limits = ctx.int8_limits()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    gpt = 1024 // p.N if p.N <= 1024 else 1
    if widths is None:
        widths = widths_grid(limits, cus, gpt, max_width)
    widths = sorted(set(int(w) for w in widths))
    cts = cggi.to_device(inputs.uniform_lwe(p, seed, max(widths)))
    out = torch.empty((max(widths), p.N + 1), dtype=torch.int32,
                      device=cts.device)
    has_ntt = time_ntt and "ntt" in ctx.forms
    times, forms, winners = {}, {}, []
    try:
        for w in widths:
            x = cts[:w]
            ref = None
            f = {}
            if has_ntt:
                f["ntt"] = round(_time(ctx, "ntt", x, out[:w], reps), 4)
                ref = out[:w].clone()
            row = {}
            for kind in cggi.KINDS:
                if limits[kind] < w:
                    continue
                _force(ctx, kind, limits)
                row[kind] = round(_time(ctx, "int8", x, out[:w], reps), 4)
                if ref is None:
                    ref = out[:w].clone()
                elif not torch.equal(out[:w], ref):
                    raise RuntimeError(f"tune: kernel {kind} at width {w} "
                                       "disagrees with the reference outputs")
            best = min(row, key=row.get)
            winners.append((w, best))
            times[str(w)] = row
            f["int8"] = row[best]
            forms[str(w)] = f
    finally:
        ctx.int8_plan(None)
    return {"params": p.name, "device": torch.cuda.get_device_name(0),
            "cus": cus, "limits": limits, "widths": widths, "reps": reps,
            "times": times, "forms": forms, "checked": True,
            "plan": plan_from_winners(winners)}


def apply(ctx, table):
    """Install the table's int8 plan on the context."""
    ctx.int8_plan([(k, int(c)) for k, c in table["plan"]])


def load_or_tune(ctx, p, path=None, **kw):
    """The cached table for this parameter set, device and build, tuned and
    written first if absent."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    key = cache_key(p, torch.cuda.get_device_name(0), cus)
    if path is None:
        path = os.path.join(cache_dir(), key + ".json")
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
        if table.get("key") == key and table.get("checked"):
            return table
    table = autotune(ctx, p, **kw)
    ctx.check()            # no latency-mode time-out since the timings
    table["key"] = key
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1)
    os.replace(tmp, path)
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--params", default="default", choices=list(params.ALL))
    ap.add_argument("--max-width", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None,
                    help="JSON path (default: the cache entry)")
    ap.add_argument("--seed", type=int, default=1)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("tune: no GPU visible (the library runs on HIP "
                         "devices only)")
    p = params.ALL[a.params]
    bsk, ksk = inputs.uniform_keys(p, a.seed)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    table = load_or_tune(ctx, p, path=a.out, reps=a.reps,
                         max_width=a.max_width, seed=a.seed)
    print(json.dumps({"key": table["key"], "plan": table["plan"],
                      "limits": table["limits"]}))
    for w in table["widths"]:
        print(json.dumps({"width": w, "int8": table["times"][str(w)],
                          "forms": table["forms"][str(w)]}))
    ctx.close()


if __name__ == "__main__":
    main()
