"""CPU FP64 oracle for block-filtered exchange-correlation (EXC) integration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links or executes this
package: only the test suite, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code with the HIP library (no kernels, headers, helpers, tables or generators); the two
meet only through the seeded inputs of the ``synth`` package.

It is a plain, slow, obviously-correct transcription of what the paper defines:

* ``basis``       Phi_{mu i} = chi_mu(r_i) (Sec. II-A, eq. phi_def; Appendix A "Gaussian basis
                  functions") and its gradient.
* ``functionals`` LDA Slater exchange; PBE exchange + PW92/PBE correlation (published forms).
* ``exc``         the dense definition: R = D Phi (eq. r_equals_dphi), rho_i = sum_mu Phi X
                  (Appendix A "The density matrix"), E_xc = sum_i w_i f_i, and
                  F^xc = b Phi W Phi^T (eq. fxc_matrix_form) generalised to GGA as V = M + M^T.
* ``reorder``     atom grouping + Morton (Z-order) grid ordering (Sec. III-B.2, eq. morton_code).
* ``addressing``  parallel addressing by exclusive prefix sum (Appendix D, Alg. parallel_where).
* ``blocked``     the block-filtered method literally: block summaries and retention
                  (eqs. block_summary_A .. retained_blocks_B), intersections (eq. block_intersection),
                  executable pairs (eqs. block_pair_filter, executed_block_pairs) and the executed sums
                  (eq. executed_block_output).

Every floating-point step is FP64.  Readings of points the paper leaves open are listed in the
module that takes them.
"""
from . import addressing, basis, blocked, exc, functionals, reorder  # noqa: F401
from .exc import eval_exc, rho_at_points  # noqa: F401
from .blocked import eval_blocked  # noqa: F401
