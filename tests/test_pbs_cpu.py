"""Programmable bootstrapping on the CPU: the lookup-table test polynomial
(paper_2306_11006_amd.pbs) run through the oracle's bootstrap and key
switch with real toy keys must return f(m) for every message m, for 1-, 2-
and 3-bit messages and several tables (this pins the table construction:
its boxes, their centring and the negacyclic wrap of message 0)."""
import numpy as np
import pytest

from conftest import real_keys
from paper_2306_11006_amd import inputs, params, pbs

TABLES = {
    "identity": lambda p: list(range(p)),
    "negate": lambda p: [(-m) % p for m in range(p)],
    "square": lambda p: [(m * m) % p for m in range(p)],
    "random": lambda p: inputs.rng(900 + p).integers(0, p, size=p).tolist(),
}


def test_encode_decode_round_trip():
    for p_msg in (2, 4, 8, 16):
        d = pbs.delta(p_msg)
        assert d * 2 * p_msg == 1 << 32
        for m in range(p_msg):
            ph = pbs.encode(m, p_msg)
            for err in (0, d // 2 - 1, -(d // 2 - 1)):
                assert pbs.decode((ph + err) % (1 << 32), p_msg) == m
                assert pbs.decode((ph + err) % (1 << 32), p_msg, True) == m
            assert pbs.decode((ph + (1 << 31)) % (1 << 32), p_msg,
                              True) == m + p_msg
    with pytest.raises(ValueError):
        pbs.delta(3)


def test_lut_layout():
    N, p_msg = 256, 4
    f = [3, 1, 0, 2]
    v = pbs.lut_test_vector(f, p_msg, N)
    d = pbs.delta(p_msg)
    box = N // p_msg
    assert v[0] == f[0] * d and v[box // 2 - 1] == f[0] * d
    assert v[box // 2] == f[1] * d and v[box + box // 2 - 1] == f[1] * d
    assert v[N - box // 2 - 1] == f[3] * d
    assert all(int(x) == ((1 << 32) - f[0] * d) % (1 << 32)
               for x in v[N - box // 2:])


@pytest.mark.parametrize("p_msg", [2, 4, 8])
@pytest.mark.parametrize("table", sorted(TABLES))
def test_lut_bootstrap_oracle(O, p_msg, table):
    p = params.TOY
    keys = real_keys(p, 3)
    f = TABLES[table](p_msg)
    v = pbs.lut_test_vector(f, p_msg, p.N)
    draws = inputs.encryption_draws(p, 910 + p_msg, p_msg)
    for m in range(p_msg):
        ct = O.lwe_encrypt(keys["s"], draws["a"][m], draws["e"][m],
                           pbs.encode(m, p_msg))
        big = O.bootstrap(p, keys["bsk"], ct, v)
        assert pbs.decode(O.lwe_phase(keys["K"], big), p_msg, True) == \
            f[m], (table, p_msg, m)
        small = O.keyswitch(p, keys["ksk"], big)
        assert pbs.decode(O.lwe_phase(keys["s"], small), p_msg, True) == \
            f[m], (table, p_msg, m)


@pytest.mark.parametrize("p_msg", [2, 4, 8])
def test_lut_box_edges(O, p_msg):
    """Every message encrypted with noise +-delta/4 (a quarter box off the
    centre; -delta/4 on m = 0 lands in the wrap region phi~ in [N, 2N)) is
    still mapped to f(m)."""
    p = params.TOY
    keys = real_keys(p, 3)
    f = [(3 * m + 1) % p_msg for m in range(p_msg)]     # f(0) != 0
    v = pbs.lut_test_vector(f, p_msg, p.N)
    d = pbs.delta(p_msg)
    draws = inputs.encryption_draws(p, 920 + p_msg, 2 * p_msg)
    for m in range(p_msg):
        for k, err in enumerate((-(d // 4), d // 4)):
            ct = O.lwe_encrypt(keys["s"], draws["a"][2 * m + k], err,
                               pbs.encode(m, p_msg))
            big = O.bootstrap(p, keys["bsk"], ct, v)
            # the padding bit must come out clear, so a wrong sign of the
            # wrapped box shows even where -f(0) = f(0) mod p
            assert pbs.decode(O.lwe_phase(keys["K"], big), p_msg, True) == \
                f[m], (p_msg, m, err)


def _mutant_no_centring(f, p_msg, N):
    table = [int(f(m)) if callable(f) else int(f[m]) for m in range(p_msg)]
    box = N // p_msg
    return np.array([(table[j // box] % p_msg) * pbs.delta(p_msg)
                     for j in range(N)], dtype=np.uint64).astype(np.uint32)


def _mutant_wrap_not_negated(f, p_msg, N, _orig=pbs.lut_test_vector):
    v = _orig(f, p_msg, N).astype(np.int64)
    table = [int(f(m)) if callable(f) else int(f[m]) for m in range(p_msg)]
    v[N - (N // p_msg) // 2:] = (table[0] % p_msg) * pbs.delta(p_msg)
    return v.astype(np.uint32)


@pytest.mark.parametrize("mutant", [_mutant_no_centring,
                                    _mutant_wrap_not_negated])
@pytest.mark.parametrize("p_msg", [2, 4])
def test_box_edge_pin_catches_planted_mistake(O, monkeypatch, mutant, p_msg):
    monkeypatch.setattr(pbs, "lut_test_vector", mutant)
    with pytest.raises(AssertionError):
        test_lut_box_edges(O, p_msg)
