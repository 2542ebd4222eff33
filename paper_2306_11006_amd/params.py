"""CGGI parameter sets used by the library, its tests and its benchmark.

Plain numbers only.  The names describe the workload each set serves:

* ``TOY``     -- n=128, N=256, Bg=2^8 l=2, KS base 2^2 t=6, noise 2^-25;
* ``DEFAULT`` -- n=630, N=1024, Bg=2^7 l=3, KS base 2^2 t=8, LWE noise
  2^-15, TRGSW noise 2^-25 (the 128-bit-class TFHE shape the paper's
  Section 2.2 describes: 630-coefficient LWE, 1024-coefficient TLWE);
* ``LARGE``   -- n=742, N=2048, Bg=2^10 l=2, KS base 2^3 t=5.

Noise is given as log2 of the inverse standard deviation on the torus
(sigma = 2^-x).  The paper's own experiments (Section 6) use n=512 with
LWE noise 2^-15 and N=1024; the sizes here are the ones the library is
measured on.
"""
from dataclasses import dataclass


@dataclass(frozen=True)
class Params:
    name: str
    n: int            # LWE dimension (number of CMux steps)
    N: int            # TRLWE ring degree, X^N + 1
    k: int            # TRLWE mask polynomials (always 1 here)
    bg_bit: int       # log2 of the gadget base Bg
    l: int            # gadget levels
    ks_base_bit: int  # log2 of the key-switch base
    ks_t: int         # key-switch levels
    lwe_noise_log2: int  # LWE / key-switching key noise std = 2^-x
    bk_noise_log2: int   # bootstrapping key noise std = 2^-x

    @property
    def ks_base(self) -> int:
        return 1 << self.ks_base_bit

    @property
    def bsk_shape(self):
        return (self.n, 2 * self.l, 2, self.N)

    @property
    def ksk_shape(self):
        return (self.N, self.ks_t, self.ks_base, self.n + 1)

    def as_tuple(self):
        return (self.n, self.N, self.k, self.bg_bit, self.l,
                self.ks_base_bit, self.ks_t)


TOY = Params("toy", n=128, N=256, k=1, bg_bit=8, l=2, ks_base_bit=2, ks_t=6,
             lwe_noise_log2=25, bk_noise_log2=25)
DEFAULT = Params("default", n=630, N=1024, k=1, bg_bit=7, l=3, ks_base_bit=2,
                 ks_t=8, lwe_noise_log2=15, bk_noise_log2=25)
LARGE = Params("large", n=742, N=2048, k=1, bg_bit=10, l=2, ks_base_bit=3,
               ks_t=5, lwe_noise_log2=15, bk_noise_log2=30)

ALL = {p.name: p for p in (TOY, DEFAULT, LARGE)}
