"""MI355X-native simplex-in-cell (SIC) 1D1V Vlasov-Poisson step.

The compute path lives in ``libsic.so`` (hand-written HIP kernels for gfx950
behind a C ABI declared in ``include/sic.h``).  ``binding`` marshals arguments
into that library; ``inputs`` builds seeded synthetic initial conditions.
Nothing is loaded at import time, so the input generators can be used on a
machine without the library.
"""

__all__ = ["binding", "inputs", "serve"]
