"""FP64 CPU oracle for the shearlet-regularised multi-label segmentation ADMM.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of what Haeuser & Steidl, "Convex Multiclass Segmentation with
Shearlet Regularization" (arXiv 1112.1805) compute: the Meyer-type building
blocks and the cone-adapted, translation-invariant finite discrete shearlet
transform of Section 2, the convex multi-label model and its ADMM of Section 3, and
the primal-dual iteration the paper names as the alternative at the end of Section 3, and
the TV and nonlocal comparison models of Section 4.
Everything is float64 numpy / scipy.fft, with no blocking, fusion
or reordering beyond what the paper's definitions state.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library (``paper_1112_1805_amd``)
and never imports it.

Readings taken where the paper is silent or garbled (see each function):

* frequency scaling rho = 4**J / N, so the top grid frequency lands on the end
  of the J-scale radial partition (exactly the paper's integer grid when
  N = 4**J);
* even-N Nyquist bins get the energy-symmetrised filter value
  sqrt((psi(w)^2 + psi(-w)^2)/2), which keeps the Parseval identity and makes
  every coefficient image real;
* zero initial ADMM state, fixed iteration count, thresholds gamma*lambda_scale
  with the low-pass using lambda_0.

Parity status: every function here is pinned by tests/test_oracle_*.py against
closed forms, identities (Lemma 2.1, the scaling-function overlap identity,
Theorem 2.2), a naive DFT, brute-force simplex projection and the ADMM
optimality conditions.  The segmentation quality against the paper's figures
is parity unpinned (the images are not published).
"""
from .meyer import meyer_v, meyer_b, psi1_hat, psi2_hat, phi_1d
from .filters import freq_index, filter_list, num_filters, filter_bank, filter_scale_index
from .transform import fft2, ifft2, naive_dft2, forward, adjoint, denoise
from .prox import soft_shrink, project_simplex, project_simplex_paper, project_simplex_bruteforce
from .model import datacost, lambda_per_filter, admm, energy, labels_of, AdmmResult
from .primaldual import primal_dual, dual_value, PdResult
from .nlmodel import nl_graph, window_distances, patch_distance, gaussian_patch, apply_D, apply_Dt, nl_tv, nl_energy, nl_primal_dual, NlResult
from .tvmodel import grad, grad_adjoint, tv, tv_energy, solve_identity_plus_laplacian, group_shrink, tv_admm, TvResult

__all__ = [
    "meyer_v", "meyer_b", "psi1_hat", "psi2_hat", "phi_1d",
    "freq_index", "filter_list", "num_filters", "filter_bank", "filter_scale_index",
    "fft2", "ifft2", "naive_dft2", "forward", "adjoint", "denoise",
    "soft_shrink", "project_simplex", "project_simplex_paper", "project_simplex_bruteforce",
    "datacost", "lambda_per_filter", "admm", "energy", "labels_of", "AdmmResult",
    "primal_dual", "dual_value", "PdResult",
    "grad", "grad_adjoint", "tv", "tv_energy", "solve_identity_plus_laplacian", "group_shrink", "tv_admm",
    "TvResult",
    "nl_graph", "window_distances", "patch_distance", "gaussian_patch", "apply_D", "apply_Dt", "nl_tv",
    "nl_energy", "nl_primal_dual", "NlResult",
]
