"""Full-size expected outputs of the gate workloads, as per-row digests.

Test infrastructure.  Each case below is a seeded workload at the default
parameter set (n=630, N=1024, Bg=2^7 l=3, key switch base 2^2 t=8); its
expected output rows are computed by the CPU oracle alone (``oracle/``:
schoolbook negacyclic products, the gate steps of Section 2.2 / Fig. 1) and
stored as one truncated SHA-256 digest per row in ``<case>.digests``.  The
GPU tests build the same inputs from the same seeds, run the HIP library,
hash every output row the same way and compare row by row, so every output
coefficient of the full-size launch is checked against the oracle without
running the oracle on the GPU machine.

Running this file (``python tests/golden/digests.py [case ...]``) rewrites
the digest files.  It imports only the oracle and the seeded input
generators; nothing here calls the HIP library.  The largest case takes
about two hours of eight host cores.

Cases:
  level1024_nand_uniform  1024 independent NAND gates, uniform keys (seed
                          2306) and uniform input ciphertexts (seed 2307):
                          the benchmark's level; rows = the 1024 output
                          wires in gate order.
  level1024_nand_keygen   1024 NAND gates with oracle-generated keys (key
                          draws seed 1) on 2048 fresh encryptions of random
                          bits (seed 2310); rows = the 1024 output wires.
  adder_mult16_keygen     a 16-bit ripple-carry adder beside a 16x16 array
                          multiplier (1455 gates, 88 levels), keys as above,
                          random operands (seed 620); rows = every wire.
  mixed16384_uniform      16,384 independent gates with opcodes uniform
                          over NAND/AND/OR/XOR/MUX (seed 78), uniform keys
                          (seed 77) and inputs (seed 79); rows = the 16,384
                          output wires.
"""
import concurrent.futures as cf
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2306_11006_amd import inputs, params  # noqa: E402

MU = 1 << 29
DIGEST_HEX = 16          # 64-bit prefix of the SHA-256 of each row
CASES = ("level1024_nand_uniform", "level1024_nand_keygen",
         "adder_mult16_keygen", "mixed16384_uniform")


def row_digests(rows):
    """Truncated SHA-256 of each row's little-endian uint32 bytes."""
    a = np.ascontiguousarray(rows, dtype="<u4")
    return [hashlib.sha256(r.tobytes()).hexdigest()[:DIGEST_HEX] for r in a]


def _encode(bit):
    return MU if bit else (1 << 32) - MU


def _keygen(O, p, seed):
    d = inputs.key_draws(p, seed)
    bsk = O.make_bsk(p, d["s"], d["K"], d["bsk_a"], d["bsk_e"])
    ksk = O.make_ksk(p, d["s"], d["K"], d["ksk_a"], d["ksk_e"])
    return dict(s=d["s"], K=d["K"], bsk=bsk, ksk=ksk)


def _encrypt(O, p, s, bits, seed):
    d = inputs.encryption_draws(p, seed, len(bits))
    return np.stack([O.lwe_encrypt(s, d["a"][i], d["e"][i], _encode(b))
                     for i, b in enumerate(bits)])


def nand_gates(G):
    """NAND gate g reads wires 2g, 2g+1 and writes wire 2G + g."""
    idx = np.arange(G, dtype=np.int32)
    z = np.zeros(G, np.int32)
    return np.stack([z, 2 * idx, 2 * idx + 1, z, 2 * G + idx],
                    axis=1).astype(np.int32)


def build(name, O):
    """Inputs of a case: dict with p, bsk, ksk, gates [G, 5] in a valid
    sequential order, wires [W, n+1] (initial values) and rows (indices of
    the wires whose final values the digests cover).  Cases with real keys
    also carry s (the LWE key) and a check of the decrypted outputs."""
    p = params.DEFAULT
    if name == "level1024_nand_uniform":
        G = 1024
        bsk, ksk = inputs.uniform_keys(p, 2306)
        wires = inputs.uniform_lwe(p, 2307, 3 * G)
        return dict(p=p, bsk=bsk, ksk=ksk, gates=nand_gates(G), wires=wires,
                    rows=np.arange(2 * G, 3 * G))
    if name == "level1024_nand_keygen":
        G = 1024
        k = _keygen(O, p, 1)
        bits = inputs.rng(2311).integers(0, 2, size=2 * G)
        wires = np.zeros((3 * G, p.n + 1), dtype=np.uint32)
        wires[: 2 * G] = _encrypt(O, p, k["s"], bits, 2310)
        want = 1 - (bits[0::2] & bits[1::2])
        return dict(p=p, bsk=k["bsk"], ksk=k["ksk"], s=k["s"],
                    gates=nand_gates(G), wires=wires,
                    rows=np.arange(2 * G, 3 * G), plain=want)
    if name == "adder_mult16_keygen":
        k = _keygen(O, p, 1)
        nl, io = inputs.adder_multiplier_circuit(16)
        g = inputs.rng(620)
        A, B, X, Y = (int(v) for v in g.integers(0, 1 << 16, size=4))
        bits = {}
        for nm, val in zip("abxy", (A, B, X, Y)):
            for i, w in enumerate(io[nm]):
                bits[w] = (val >> i) & 1
        wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
        ins = sorted(bits)
        wires[ins] = _encrypt(O, p, k["s"], [bits[w] for w in ins], 621)
        return dict(p=p, bsk=k["bsk"], ksk=k["ksk"], s=k["s"],
                    gates=nl.array(), wires=wires,
                    rows=np.arange(nl.n_wires), io=io,
                    operands=(A, B, X, Y))
    if name == "mixed16384_uniform":
        G = 16384
        bsk, ksk = inputs.uniform_keys(p, 77)
        wires = np.zeros((4 * G, p.n + 1), dtype=np.uint32)
        wires[: 3 * G] = inputs.uniform_lwe(p, 79, 3 * G)
        return dict(p=p, bsk=bsk, ksk=ksk, gates=inputs.random_gate_batch(78, G),
                    wires=wires, rows=np.arange(3 * G, 4 * G))
    raise KeyError(name)


def depths(gates, n_wires):
    """Depth of every gate of a netlist given in a valid sequential order:
    1 + the deepest gate writing one of its inputs (circuit inputs: 0)."""
    depth_of_wire = np.zeros(n_wires, dtype=np.int64)
    out = np.empty(len(gates), dtype=np.int64)
    n_in = {0: 2, 1: 2, 2: 2, 3: 2, 4: 3, 5: 1, 6: 1, 7: 0, 8: 0, 9: 2,
            10: 2}
    for i, (op, a, b, c, o) in enumerate(np.asarray(gates).tolist()):
        used = (a, b, c)[: n_in[op]]
        d = 1 + max((depth_of_wire[w] for w in used), default=0)
        depth_of_wire[o] = d
        out[i] = d
    return out


def oracle_run(O, case, threads, log=None):
    """Final wire values of a case computed by the oracle: gates of equal
    depth are independent and run on a thread pool, depths in order."""
    p, bsk, ksk = case["p"], case["bsk"], case["ksk"]
    w = case["wires"].copy()
    gates = case["gates"]
    dep = depths(gates, len(w))

    def one(i):
        op, a, b, c, o = (int(v) for v in gates[i])
        return o, O.gate(p, op, bsk, ksk, w[a], w[b], w[c])

    t0 = time.time()
    done = 0
    with cf.ThreadPoolExecutor(threads) as ex:
        for d in range(1, int(dep.max()) + 1 if len(dep) else 1):
            idx = np.nonzero(dep == d)[0]
            for lo in range(0, len(idx), 256):
                for o, val in ex.map(one, idx[lo: lo + 256]):
                    w[o] = val
                done += len(idx[lo: lo + 256])
                if log:
                    log(f"  {done}/{len(gates)} gates, "
                        f"{time.time() - t0:.0f} s")
    return w


def path(name):
    return os.path.join(HERE, name + ".digests")


def load(name):
    """Stored digests of a case: list of hex strings, one per row."""
    rows = []
    with open(path(name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


def compare(name, got_rows):
    """Indices of the rows whose digest differs from the stored one."""
    want = load(name)
    got = row_digests(got_rows)
    if len(got) != len(want):
        raise AssertionError(f"{name}: {len(got)} rows, {len(want)} stored")
    return [i for i, (a, b) in enumerate(zip(got, want)) if a != b]


def write(name, threads):
    import oracle as O
    O.lib()
    case = build(name, O)
    log = lambda m: print(f"[{name}]{m}", file=sys.stderr, flush=True)  # noqa
    t0 = time.time()
    w = oracle_run(O, case, threads, log)
    dig = row_digests(w[case["rows"]])
    hdr = [
        f"# {name}: per-row digests of the oracle's output wires",
        "# (first 16 hex digits of the SHA-256 of each row's little-endian",
        "# uint32 bytes, rows in the order the case defines); written by",
        "# tests/golden/digests.py from the CPU oracle only",
        f"# rows: {len(dig)}; oracle wall time {time.time() - t0:.0f} s "
        f"on {threads} threads",
    ]
    with open(path(name) + ".tmp", "w") as f:
        f.write("\n".join(hdr + dig) + "\n")
    os.replace(path(name) + ".tmp", path(name))
    log(f" wrote {len(dig)} digests")


def main(argv):
    threads = int(os.environ.get("DIGEST_THREADS", os.cpu_count() or 4))
    names = argv or list(CASES)
    for n in names:
        write(n, threads)


if __name__ == "__main__":
    main(sys.argv[1:])
