"""The oracle pins have teeth: plant a plausible mistake in a copy of the
oracle's C source, build it on the CPU, and check that the pin aimed at that
part fails.  (Mistakes are planted in the oracle only, never on a GPU.)"""
import ctypes
import os
import subprocess

import pytest

import oracle
from oracle import api
from paper_2306_11006_amd import params
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(api.__file__), "cggi_oracle.c")

MUTANTS = {
    # wrap-around sign of the negacyclic product dropped
    "product_sign": ("acc[m + k - N] -= xm * y[k];",
                     "acc[m + k - N] += xm * y[k];",
                     lambda O: pins.test_poly_mul_matches_folded_convolution(
                         O, 256)),
    # modulus switch truncates instead of rounding
    "modswitch_round": ("return (uint32_t)((uint32_t)(u + half) >>",
                        "return (uint32_t)((uint32_t)(u + 0) >>",
                        lambda O: pins.test_modswitch_nearest_ties_up(O, 1024)),
    # gadget decomposition without its rounding offset
    "decomp_round": ("w += 1u << (31 - l * beta);          /* rounding",
                     "w += 0u << (31 - l * beta);          /* rounding",
                     lambda O: pins.test_decomp_range_and_recomposition(
                         O, 7, 3)),
    # sample extraction with the wrong sign on the mask
    "extract_sign": ("out[j] = 0u - acc[N - j];", "out[j] = acc[N - j];",
                     lambda O: pins.test_sample_extract_identity(O)),
    # gadget rows added to the wrong component
    "trgsw_component": ("if (c == 0)\n                    mask[0] += g;",
                        "if (c == 1)\n                    mask[0] += g;",
                        lambda O: pins.test_external_product_closed_form(
                            O, params.TOY, 1)),
    # accumulator initialised with X^(+b~) instead of X^(-b~)
    "acc_init_exponent": ("(int)((2u * N - bt) % (2u * N))", "(int)bt",
                          lambda O: pins.test_blind_rotation_closed_form(
                              O, params.TOY)),
    # key-switch digits truncated
    "ks_round": ("w += 1u << (31 - t * gamma);", "w += 0u;",
                 lambda O: pins.test_keyswitch_closed_form(O, params.TOY)),
    # CMux difference taken the wrong way round
    "cmux_sub": ("tmp[c * N + j] -= acc[c * N + j];",
                 "tmp[c * N + j] += acc[c * N + j];",
                 lambda O: pins.test_cmux_closed_form(O, 1)),
    # NAND constant wrong (Enc(0) read literally as 0)
    "nand_const": ("case ORC_NAND: orc_linear(n, ORC_MU, -1, x, -1, y, lin);",
                   "case ORC_NAND: orc_linear(n, 0u, -1, x, -1, y, lin);",
                   lambda O: pins.test_gate_truth_tables_toy(O, 1)),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_catches_planted_mistake(name, tmp_path, monkeypatch):
    old, new, check = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-w",
                    "-o", str(so), str(mutated)], check=True)
    api._lib = None
    real = api.LIB
    monkeypatch.setattr(api, "LIB", str(so))
    import conftest
    saved = dict(conftest._KEYS)
    conftest._KEYS.clear()
    try:
        api.lib()
        with pytest.raises(AssertionError):
            check(oracle)
    finally:
        conftest._KEYS.clear()
        conftest._KEYS.update(saved)
        api._lib = None
        monkeypatch.setattr(api, "LIB", real)
        api.lib()
    assert isinstance(api._lib, ctypes.CDLL)


def _noise(scale_shift=0, rounding=True, uniform=False):
    import numpy as np

    def f(g, shape, x):
        if x is None:
            return np.zeros(shape, dtype=np.int32)
        z = (g.random(size=shape) - 0.5) * np.sqrt(12.0) if uniform \
            else g.standard_normal(size=shape)
        v = z * float(2 ** (32 - x - scale_shift))
        v = np.rint(v) if rounding else v
        return v.astype(np.int64).astype(np.int32)
    return f


@pytest.mark.parametrize("name,mutant", [
    ("noise scale halved", _noise(scale_shift=1)),
    ("noise truncated, not rounded", _noise(rounding=False)),
    ("noise uniform, not Gaussian", _noise(uniform=True)),
])
def test_noise_pin_catches_planted_mistake(name, mutant, monkeypatch):
    from paper_2306_11006_amd import inputs
    monkeypatch.setattr(inputs, "gaussian_i32", mutant)
    with pytest.raises(AssertionError):
        pins.test_noise_draws_are_rounded_gaussians()
