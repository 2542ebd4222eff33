"""bench.py host helpers (no GPU): the operation counts behind the roofline
figures and the stored-counter lookup behind roofline.traffic."""
import os
import shutil
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2306_11006_amd import params  # noqa: E402


def test_int8_ops_default_and_large():
    # 2 * 2N * (2lN * S) * 4 limbs * n
    assert bench.int8_ops_per_bootstrap(params.DEFAULT) == \
        2 * 2048 * (6 * 1024) * 4 * 630
    assert bench.int8_ops_per_bootstrap(params.LARGE) == \
        2 * 4096 * (4 * 2048 * 2) * 4 * 742


def test_int8_ops_karatsuba_and_kernel_lookup():
    # three half-length products: 3 * 2 * 2(N/2) * (2l(N/2) * S) * 4 * n
    full = bench.int8_ops_per_bootstrap(params.DEFAULT)
    assert bench.int8_ops_per_bootstrap(params.DEFAULT, "kara2") == \
        3 * 2 * 1024 * (6 * 512) * 4 * 630 == full * 3 // 4
    plan = [("split8", 16), ("tiles1", 256), ("tiles2", 512),
            ("kara2", 2**31 - 1)]
    assert bench.int8_kind_for(plan, 1) == "split8"
    assert bench.int8_kind_for(plan, 512) == "tiles2"
    assert bench.int8_kind_for(plan, 1024) == "kara2"
    assert bench.int8_kernel_name(params.DEFAULT, "kara2") == \
        "k_bootstrap_int8_kara<1024, 3, 1, 7>"
    assert bench.int8_kernel_name(params.TOY, "kara2") == \
        "k_bootstrap_int8_kara<256, 2, 2, 0>"
    assert bench.int8_kernel_name(params.DEFAULT, "tiles4") == \
        "k_bootstrap_int8<1024, 3, 1, 4>"
    assert bench.int8_kernel_name(params.LARGE, "tiles4") == \
        "k_bootstrap_int8<2048, 2, 2, 4>"


def test_ntt_mulmods_default():
    # (2l + 2) transforms of N/2 log2 N butterflies + 2l * 2N pointwise
    assert bench.ntt_mulmods_per_bootstrap(params.DEFAULT) == \
        630 * (8 * 512 * 10 + 6 * 2048)


def test_code_hash_ignores_comments(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f() { return 1; }\n")
    b.write_text("// header\n\nint f() { return 1; }  // trailing\n")
    assert bench.code_sha256(str(a)) == bench.code_sha256(str(b))
    b.write_text("int f() { return 2; }\n")
    assert bench.code_sha256(str(a)) != bench.code_sha256(str(b))


def test_stored_traffic_follows_the_source(tmp_path, monkeypatch):
    """Counters are reported for the kernel source they were taken on and
    dropped (None) once the code changes."""
    prof = os.path.join(ROOT, "profiles", "eval_level_1024_nand_default.md")
    text = open(prof).read()
    src_rel = [ln.split(":", 1)[1].strip() for ln in text.splitlines()
               if ln.startswith("traffic-source:")][0]
    fake = tmp_path / "repo"
    (fake / "profiles").mkdir(parents=True)
    shutil.copy(prof, fake / "profiles" / os.path.basename(prof))
    os.makedirs(fake / os.path.dirname(src_rel))
    shutil.copy(os.path.join(ROOT, src_rel), fake / src_rel)
    monkeypatch.setattr(bench, "ROOT", str(fake))
    same = bench.stored_traffic()
    with open(fake / src_rel, "a") as f:
        f.write("\nstatic int changed_kernel_code;\n")
    assert bench.stored_traffic() is None
    if same is not None:   # the committed counters match the committed kernel
        assert same > 0


def test_cpu_baseline_sample_rounds():
    """The oracle sample grows in rounds of `threads` gates until both the
    least gate count and the least wall time are met."""
    import numpy as np
    import oracle as O
    from paper_2306_11006_amd import inputs
    p = params.TOY
    bsk, ksk = inputs.uniform_keys(p, 11)
    G = 12
    wires = inputs.uniform_lwe(p, 12, 2 * G)
    gates = np.array([[0, 2 * g, 2 * g + 1, 0, 2 * G + g] for g in range(G)],
                     dtype=np.int32)
    want = np.stack([O.gate(p, 0, bsk, ksk, wires[2 * g], wires[2 * g + 1])
                     for g in range(G)])
    rate, n, wall, ok = bench.cpu_baseline(p, bsk, ksk, wires, gates, want,
                                           5, 0.0, 2)
    assert n == 6 and ok and rate > 0
    bad = want.copy()
    bad[1, 0] ^= 1
    assert not bench.cpu_baseline(p, bsk, ksk, wires, gates, bad, 1, 0.0,
                                  2)[3]
    # the whole batch when the time bound is never met
    assert bench.cpu_baseline(p, bsk, ksk, wires, gates, want, 1, 1e9,
                              4)[1] == G


def test_digest_mismatches_names_rows(tmp_path, monkeypatch):
    """bench.py's check of every output row against the oracle's stored
    digests uses the format tests/golden/digests.py writes."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import digests as D
    rows = np.arange(12, dtype=np.uint32).reshape(3, 4) * 977
    (tmp_path / "x.digests").write_text(
        "# header\n" + "\n".join(D.row_digests(rows)) + "\n")
    monkeypatch.setattr(bench, "DIGESTS", str(tmp_path))
    assert bench.digest_mismatches("x", rows) == []
    bad = rows.copy()
    bad[1, 2] ^= 1
    assert bench.digest_mismatches("x", bad) == [1]
    assert bench.digest_mismatches("x", rows[:2]) == [0, 1]
    assert bench.digest_mismatches("missing", rows) is None


def test_host_cpu_reports_counts():
    nproc, aff, model = bench.host_cpu()
    assert nproc >= 1 and 1 <= aff <= nproc
    assert model is None or isinstance(model, str)


def test_bootstrap_count_of_gates():
    import numpy as np
    from paper_2306_11006_amd import inputs
    g = inputs.random_gate_batch(78, 16384)
    # MUX counts two bootstraps, the other four opcodes one each
    assert bench.bootstraps_of(g) == 16384 + int((g[:, 0] == 4).sum())
    assert bench.bootstraps_of(g) == 19727
    nots = np.array([[5, 0, 0, 0, 1], [7, 0, 0, 0, 2]], dtype=np.int32)
    assert bench.bootstraps_of(nots) == 0
