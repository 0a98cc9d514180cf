"""CPU oracle for the HALLaR hot path — TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 numpy implementation of what the GPU library computes,
written from the cuHALLaR paper (arXiv 2505.13719).  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does, and it shares no code with the HIP path.

  operators.py  -- A~(UU^T), A~*(p~)U, the AL function and its U-gradient
                   (Section 2 eqs. AL function / Grad U Space; Section 4,
                   eq. A tilde operator; Algorithms 2-5 restated as their
                   plain definitions).
  lanczos.py    -- minimum eigenpair by Lanczos with full
                   reorthogonalisation (the eigensolver of Alg. 1 step ii,
                   which the paper leaves unspecified).
  hallar.py     -- ADAP-FISTA (App. A.1), ADAP-AIPP (App. A), the HLR loop
                   with the Frank-Wolfe certificate and step (Alg. 1) and the
                   outer augmented-Lagrangian loop with the relative
                   termination test of Section 5.1 (eq. termination2).

Every function is pinned by tests under tests/ (dense definitions, the
adjoint identity, finite differences, closed-form spectra and closed-form
SDP values); none is marked "parity unpinned".
"""
from .operators import (a_tilde, a_map, adjoint_apply, adjoint_sparse, al_value,
                        al_grad, c_l1_norm)
from .lanczos import min_eig
from .hallar import ALFunction, Options, Result, hallar, fista, aipp, fw_alpha, fw_step, metrics

__all__ = ["a_tilde", "a_map", "adjoint_apply", "adjoint_sparse", "al_value", "al_grad",
           "c_l1_norm", "min_eig", "ALFunction", "Options", "Result", "hallar", "fista", "aipp",
           "fw_alpha", "fw_step", "metrics"]
