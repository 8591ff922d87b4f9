"""FP64 CPU reference for the graph-propagation (GP) vectors of
"Scaling Up Graph Propagation Computation on Large Graphs: A Local Chebyshev
Approximation Approach" (arXiv 2412.10789).

TEST INFRASTRUCTURE ONLY.  This package is the oracle that the GPU library
is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library itself never does,
and it shares no code with the library (inputs come from ``synth``, which
holds no propagation arithmetic).

Plain and slow on purpose: every function follows one passage of the paper
in the paper's order and notation, with a library primitive (a sparse or
dense matrix product, a dense solve, a matrix exponential, an eigensolver)
as the only building blocks.  Floating point is IEEE double throughout.

Modules
  coefficients  Taylor coefficients (Def. 3, Def. 4) and Chebyshev
                coefficients (Lemma 1, Lemma 2, Lemma 3)
  truncation    coefficient tails, the truncation step K (Thm. 2 and the
                l1-certified reading), PwMethod's N from its exact tail
  propagation   P = A D^{-1}; ChebyPower (Algorithm 3); PwMethod
                (Algorithm 1); Chebyshev vectors T_k(P) e_s (Eq. 6)
  dense         dense definitions for tiny graphs: inverse (Def. 3),
                matrix exponential (Def. 4), eigen route (Lemma 1 proof),
                f(D^{-a} A D^{-b}) X (Def. 8)
  errors        error measures (Def. 5) and the PPR residual certificate
  push          ChebyPush (Alg. 4) and the subset Chebyshev recurrence
                (Def. 7), with the two threshold readings of Sec. 4
  bidirectional ChebyPush + alpha-random walks for SSPPR (Alg. 5), walks
                drawn from SplitMix64 counters
  circulant     closed forms on circulant graphs through the DFT (exact
                vectors and Algorithm 3's output at any size)
  generalized   Z = f(D^{-a} A D^{-b}) X (Def. 8) through Thm. 5: the series
                of Alg. 3 / Alg. 1 on D^{a} X, scaled by D^{-a}
  native        the same Alg. 3 / Alg. 1 in plain C with an OpenMP node
                loop (oracle/c/chebypower.c), for graphs with billions of arcs
"""

from . import bidirectional, circulant, coefficients, dense, errors, generalized, propagation, push, truncation  # noqa: F401,E501
