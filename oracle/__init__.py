"""CPU FP64 oracle for walk-based Laplacians (Arrigo & Durastante, arXiv 2601.11338).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously-correct
reference the HIP library is checked against.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product path
never does, and it shares no code with the HIP library (the only common inputs
come from the seeded generators in ``synth``, which hold none of the method's
arithmetic).

Everything is float64 numpy/scipy.  Each function names the passage of the
paper it follows.  Readings of passages where the paper is silent or
inconsistent are stated where they are used.

Pinned (see tests/test_oracle_*.py) against: brute-force walk enumeration, the
paper's worked example (Fig. 1), closed forms on regular graphs, the lemma and
propositions on symmetry / zero row sums / M-matrix structure, library routines
in the special cases that reduce to them, published Philox known-answer
vectors, and finite differences for the MLP gradients.

Parity unpinned by the paper: the learned control variate (the paper has no
learned part); its pins are internal identities (unbiasedness, exactness with a
perfect control variate) only.
"""

from . import walks, genfun, laplacian, sparse, estimators, philox, mlp  # noqa: F401
