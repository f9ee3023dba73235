"""FP64 CPU oracle for Faster Mean-shift (arXiv 2007.14283).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the GPU library (no kernels, headers, helpers or tables)
and imports nothing from it.

Modules
-------
seed_order  SplitMix64 and the Feistel permutation that fixes the seed order
            (Alg. 2's uniform random seed draw, read as a keyed permutation).
osop        Eq. 14, Eq. 15 and Eq. 19 and the seed-count controller (Sec. 3.2.2,
            Sec. 3.2.4).
meanshift   Normalisation (Eq. 1), the flat-kernel cosine step (Eq. 8, 9, 11),
            the seed iteration with early stopping (Sec. 3.2.3), window counts,
            mode pruning, coverage and pixel assignment (Alg. 2), and Alg. 1 as
            a brute-force reference for tiny inputs.
cluster     The whole of Alg. 2 under the online seed optimisation policy.
unroll      T unrolled steps from given seeds and the exact (almost everywhere)
            gradient of the result with respect to the raw embeddings.

Parity status: every function is pinned by a CPU test (see the ``tests``
folder).  Three choices are readings the paper leaves open (the tie-break order
of the mode merge, the strict gamma stop and the coverage rule); each is pinned
by hand-built cases whose outcome the reading fixes exactly.
"""
from . import seed_order, osop, meanshift, cluster, unroll  # noqa: F401
