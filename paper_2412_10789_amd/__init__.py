"""MI355X (gfx950) ChebyPower: Chebyshev power iteration for personalized
PageRank and heat-kernel PageRank vectors (arXiv 2412.10789, Alg. 3),
hand-written HIP kernels behind a C ABI (include/chebyprop.h).
"""

from .chebyprop import Graph, load  # noqa: F401
