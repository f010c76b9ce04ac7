"""FP64 CPU oracle for contraction-only block-MM (B-CoMM) and joint-MM (J-CoMM)
updates of nonnegative CP and Tucker models under beta-divergences.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the HIP library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library itself
never does, and the two share no code.

Everything is written in float64 with NumPy, following the paper step by step:

* :mod:`oracle.divergence` – the beta-divergence (Sec. 3.2, Definition of the
  beta-divergence), the objective, the weight tensors P and Q (Sec. 4.1), the
  exponent gamma(beta) (Remark on gamma), and the transforms chi_1, chi_2
  (Sec. 5.3).
* :mod:`oracle.cp` – CP reconstruction (Sec. 3.3), the contraction operator
  CPContr (Sec. 6.1), the block update (Theorem "CP block multiplicative
  update"), B-CoMM (Algorithm B-CoMM) and J-CoMM (Algorithm J-CoMM, CP inner
  update of Sec. 5.3).
* :mod:`oracle.tucker` – Tucker reconstruction (App. C, eq. tucker_entry), the
  block core / factor contractions (App. C.2) and the joint ones (App. C.3),
  B-CoMM and J-CoMM for Tucker.
* :mod:`oracle.sparse` – J-CoMM for CP at beta = 1 on COO data, accumulating
  numerators over the nonzeros only (Sec. 6.4, paragraph on sparse tensors).
* :mod:`oracle.surrogate` – the explicit joint surrogate G(Theta | Theta~)
  with all constants (App. A.4, App. B.2-B.3) and the scalar subproblems
  (App. B.5).
* :mod:`oracle.unfolding` – the classical unfolding / Khatri-Rao (MTTKRP) form
  of the same updates (Sec. 7, baseline 1), an independent route used only to
  cross-check the contraction forms on tiny tensors.
* :mod:`oracle.loops` – explicit-loop forms for tiny tensors.

Readings of points the paper leaves open (values of eps and eps_X, where the
reconstruction is clipped, 0 log 0, gamma at the boundary cases, Tucker block
order, where eps is enforced in the inner loop) are fixed by keyword defaults
documented on each function.
"""
from .divergence import (beta_divergence, objective, gamma, powers,
                         chi1, chi2, EPS_DEFAULT)
from . import cp, tucker, sparse, surrogate, unfolding, loops

__all__ = [
    "beta_divergence", "objective", "gamma", "powers", "chi1", "chi2",
    "EPS_DEFAULT", "cp", "tucker", "sparse", "surrogate", "unfolding", "loops",
]
