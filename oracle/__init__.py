"""CPU oracle for the randomized minimal-norm solver (Tygert, arXiv 0905.4745).

TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 (and extended-precision) numpy /
scipy code that states what the GPU path computes.  Only the test suite, the
package's smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does, and this package imports nothing from the product.

Modules
  transforms  -- DFT matrix (eq. DFT), orthonormal Hartley matrix, SRFT matrix
                 T = S F D (eqs. SRFT, SRFT2), sketch S = T A* (eq. randmat),
                 adjoint application c = T* z (eq. nonminnorm); the optional
                 H = Theta Pi Z Theta~ Pi~ Z~ factor (eq. Rokhlin_trans).
  householder -- unblocked Householder QR (Step 2's factorisation).
  pcg         -- Step 4 read as preconditioned CG on A A* y = b with the
                 sketch's R as preconditioner, and its stopping rules.
  classical   -- the classical QR-based minimal-norm solver (Section 1 and
                 Section 7's direct method) and an extended-precision refined
                 variant.
  randomized  -- the five steps of Section 4 end to end, with intermediates.
  draws       -- the SRFT's phases and indices as the library draws them
                 (Philox4x32-10 counters, Floyd's sampling), for tests.
"""

from .transforms import (  # noqa: F401
    dft_matrix,
    fft_ortho,
    dht_matrix,
    dht_ortho,
    srft_matrix,
    srft_real_matrix,
    sketch,
    sketch_real,
    srft_adjoint,
    srft_real_adjoint,
    givens_chain_matrix,
    rokhlin_h_apply,
    rokhlin_h_matrix,
)
from .householder import householder_qr, apply_qh, normalize_r  # noqa: F401
from .pcg import pcg_minnorm, stop_threshold  # noqa: F401
from .classical import classical_minnorm, refined_minnorm, residuals_longdouble  # noqa: F401
from .randomized import randomized_minnorm  # noqa: F401
from .draws import philox4x32_10, draw_phases, draw_indices, draw_srft  # noqa: F401
