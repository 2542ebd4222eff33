import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (runs the HIP library on cuda:0)")
    config.addinivalue_line(
        "markers", "slow: long CPU test (oracle at default sizes)")


MU = 1 << 29


def signed(x):
    """uint32 torus value(s) -> signed int64."""
    x = np.asarray(x, dtype=np.int64)
    return np.where(x >= 1 << 31, x - (1 << 32), x)


def encode(bit):
    return MU if bit else (1 << 32) - MU


@pytest.fixture(scope="session")
def O():
    import oracle
    oracle.lib()
    return oracle


_KEYS = {}


def real_keys(p, seed=1):
    """Oracle-generated bsk/ksk for parameter set p (cached per session)."""
    key = (p.name, seed)
    if key not in _KEYS:
        import oracle
        from paper_2306_11006_amd import inputs
        d = inputs.key_draws(p, seed)
        bsk = oracle.make_bsk(p, d["s"], d["K"], d["bsk_a"], d["bsk_e"])
        ksk = oracle.make_ksk(p, d["s"], d["K"], d["ksk_a"], d["ksk_e"])
        _KEYS[key] = dict(s=d["s"], K=d["K"], bsk=bsk, ksk=ksk)
    return _KEYS[key]


def encrypt_bits(p, keys, bits, seed):
    """Fresh LWE encryptions of ``bits`` under keys['s'] (oracle)."""
    import oracle
    from paper_2306_11006_amd import inputs
    d = inputs.encryption_draws(p, seed, len(bits))
    return np.stack([oracle.lwe_encrypt(keys["s"], d["a"][i], d["e"][i],
                                        encode(b))
                     for i, b in enumerate(bits)])
