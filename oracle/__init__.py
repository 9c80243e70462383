"""Plain FP64 CPU oracle for the line-DG hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import, call or execute anything in this
package; the GPU library never does, and this package never imports it.  Every
function restates the paper's definitions (sections, equations and tables are
cited in each module) with dense torch/numpy operations in float64 on the CPU.
"""
from .basis import LineOps, gll_nodes, gauss_legendre, n_gauss  # noqa: F401
from .physics import Physics, EQ_POISSON, EQ_EULER, EQ_NS  # noqa: F401
from .linedg import LineDG  # noqa: F401
