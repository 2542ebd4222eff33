"""CPU oracle for batched CGGI gate bootstrapping -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps the plain C implementation in
``cggi_oracle.c`` (schoolbook negacyclic products, ArctyrEX Section 2.2 and
Fig. 1) with numpy marshalling and shares no code with the GPU library.
"""
from .api import *  # noqa: F401,F403
