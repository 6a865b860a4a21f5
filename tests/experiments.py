"""The synthetic experiments of Section 4 (E1 rank-1 streaming, E2 the
effect of k, E3 structural growth) on this repository's factor generator,
shared by the oracle's and the engine's sanity-band tests.  The paper's own
generator is not specified, so its values serve as qualitative bands."""
from synth import FactorStream, ENTRY, ROW, COL

E1_CHECK = 250      # checkpoint spacing of the rank-1 runs


def e1_stream(n_updates=10000, noise=0.0):
    """50 x 40 of rank 5 (exactly, without noise), rank-1 updates delta ~ N(0, 0.05^2).
    E2's k-sweep takes noise 0.1, so that every k is within the numerical
    rank; on the exact matrix a k above 5 keeps rank 5 (both sides)."""
    fs = FactorStream(seed=5, stream=0, n0=40, K=5, noise=noise)
    A0 = fs.initial(50)
    return A0, fs.materialize([ENTRY] * n_updates, m0=50, delta_std=0.05)


def e3_stream(n_events=100):
    """150 x 40 from a rank-6 model with noise, rows and columns appended in turn."""
    fs = FactorStream(seed=7, stream=0, n0=40, K=6, noise=0.1)
    A0 = fs.initial(150)
    return A0, fs.materialize([ROW if q % 2 == 0 else COL for q in range(n_events)], m0=150)
