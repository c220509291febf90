"""FP64 CPU oracle for Geodesic Sinkhorn -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct numpy/scipy code in float64 that computes what
the paper defines: the common kNN affinity graph and its combinatorial
Laplacian (Sec. "Heat Diffusion on a Graph"; Sec. "Geodesic Sinkhorn
Distances"), the Chebyshev/Bessel expansion of the heat kernel (Sec.
"Chebyshev Polynomials"), Algorithm 1 (Geodesic Sinkhorn), the fixed-support
barycenter (Sec. "Interpolation with discrete support"), and a hand-written
reverse-mode gradient of Algorithm 1's output.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: it imports
nothing from the library package and the library never imports it.  The only
module both sides use is ``synth`` (seeded random inputs, no method
arithmetic).

Readings of points the paper leaves silent or garbled are documented in each
function; the same list is kept with the design notes.
"""
from . import graph, heat, spectrum, sinkhorn, closed_forms, families, pairwise  # noqa: F401
