"""Host logic of the autotuner: width grid, compression of per-width winners
into a kernel plan (the rules cggi_ctx_int8_plan enforces), form choice by
width, and the cache key.  No GPU call."""
import pytest

from paper_2306_11006_amd import cggi, params, tune

LIMITS = {"split8": 32, "split4": 64, "split2": 128, "tiles1": 2**31 - 1,
          "tiles2": 2**31 - 1, "tiles4": 2**31 - 1}


def valid(plan, limits=LIMITS):
    caps = [c for _, c in plan]
    assert all(a < b for a, b in zip(caps, caps[1:]))
    assert caps[-1] >= 1 << 24
    assert not plan[-1][0].startswith("split")
    for k, c in plan:
        assert k in cggi.KINDS and 1 <= c <= limits[k]


def test_grid_holds_powers_and_boundaries():
    g = tune.widths_grid(LIMITS, cus=256, gpt=1, max_width=4096)
    assert g == sorted(set(g))
    for w in (1, 2, 32, 33, 64, 65, 128, 129, 256, 257, 512, 513, 1024,
              1025, 4096):
        assert w in g, w
    assert max(g) == 4096
    g4 = tune.widths_grid(LIMITS, cus=256, gpt=4, max_width=300)
    assert max(g4) == 300 and {64, 65, 128, 129, 256} <= set(g4)


def test_plan_from_winners_merges_runs():
    win = [(1, "split4"), (2, "split4"), (64, "split4"), (65, "split2"),
           (128, "split2"), (129, "tiles1"), (256, "tiles1"),
           (257, "tiles2"), (512, "tiles2"), (513, "tiles4"),
           (4096, "tiles4")]
    plan = tune.plan_from_winners(win)
    assert plan == [("split4", 64), ("split2", 128), ("tiles1", 256),
                    ("tiles2", 512), ("tiles4", 2**31 - 1)]
    valid(plan)


def test_plan_from_winners_edge_cases():
    # a latency-mode winner at the top of the grid gets a catch-all entry
    plan = tune.plan_from_winners([(1, "split4"), (64, "split4")])
    assert plan == [("split4", 64), ("tiles4", 2**31 - 1)]
    valid(plan)
    # non-monotone winners stay separate entries, caps still increasing
    plan = tune.plan_from_winners([(1, "tiles1"), (2, "split4"),
                                   (4, "tiles1")])
    assert plan == [("tiles1", 1), ("split4", 2), ("tiles1", 2**31 - 1)]
    valid(plan)
    assert tune.plan_from_winners([]) == [("tiles4", 2**31 - 1)]


def test_best_form_by_width():
    table = {"forms": {"1": {"int8": 3.0, "ntt": 15.0},
                       "1024": {"int8": 23.0, "ntt": 41.0},
                       "2048": {"int8": 50.0, "ntt": 45.0}}}
    assert tune.best_form(table, 1) == "int8"
    assert tune.best_form(table, 500) == "int8"      # rounds up to 1024
    assert tune.best_form(table, 1500) == "ntt"      # rounds up to 2048
    assert tune.best_form(table, 10**6) == "ntt"     # beyond the grid
    assert tune.best_form({}, 7) == "int8"
    assert tune.best_form({"forms": {"4": {"int8": 1.0}}}, 3) == "int8"


def test_cache_key_names_params_device_and_build():
    k = tune.cache_key(params.DEFAULT, "AMD Instinct MI355X", 256)
    assert k.startswith("default-n630-N1024-bg7-l3-ks2x8-AMD-Instinct-MI355X-"
                        "256cu-")
    assert k == tune.cache_key(params.DEFAULT, "AMD Instinct MI355X", 256)
    assert k != tune.cache_key(params.LARGE, "AMD Instinct MI355X", 256)


def test_tune_cli_needs_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(SystemExit, match="no GPU"):
        tune.main(["--params", "toy"])


def test_dag_cli_needs_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2306_11006_amd import dag
    with pytest.raises(SystemExit, match="no GPU"):
        dag.main(["--gates", "10"])


def test_plan_from_winners_keeps_at_most_eight_entries():
    # noisy alternation between two kernels of similar speed
    kinds = ("split8", "split4", "split2", "tiles1", "tiles2", "tiles4")
    win, w = [], 1
    for k in range(40):
        win.append((w, kinds[k % 6]))
        w += 1 + k
    # every winner respects its kind's limit, as the tuner's would
    win = [(w, k if LIMITS[k] >= w else "tiles2") for w, k in win]
    plan = tune.plan_from_winners(win)
    assert len(plan) <= 8, plan
    valid(plan)
    # a strict alternation of two throughput kernels
    alt = [(w, "tiles1" if i % 2 else "tiles2")
           for i, w in enumerate(range(200, 230))]
    plan = tune.plan_from_winners(alt)
    assert len(plan) <= 8
    valid(plan)
    # every width still goes to a kernel whose limit holds it
    for w, _ in win:
        k = next(k for k, c in plan if w <= c)
        assert LIMITS[k] >= w
    # short plans are untouched
    short = [(1, "split8"), (16, "split8"), (17, "split4"), (64, "split4"),
             (65, "tiles4")]
    assert tune.plan_from_winners(short) == [
        ("split8", 16), ("split4", 64), ("tiles4", 2**31 - 1)]
