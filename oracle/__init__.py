"""FP64 CPU oracle for phylogenetic log-likelihoods and branch-length gradients.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import,
call or link this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.

What it computes (the paper states these only in words, so the textbook
definitions are written out):

* Felsenstein's pruning algorithm for post-order partial likelihoods
  (Introduction; the paper cites Felsenstein 1981);
* the likelihood at the root as frequencies times root partials, mixed over
  rate categories, and the pattern-weighted sum of site log-likelihoods;
* pre-order partial likelihoods and the identity that the likelihood is the
  inner product of pre- and post-order partials at every node (Key
  Improvements, Algorithmic advances; Ji et al. 2020);
* the gradient with respect to every branch length as a pre . Q . post
  "sandwich" in one pre-order traversal (Discussion);
* the gradient with respect to every rate-matrix entry, with the derivative of each
  transition matrix taken to first order (Key Improvements, Algorithmic advances;
  random-effects substitution models), in ``rate_gradient.py``.

Parity pins: each function is checked in ``tests/test_oracle_*.py`` against
closed forms, brute-force summation, invariants and finite differences.
"""
from .pruning import (
    transition_matrices, tip_partials, post_order, root_site_loglik, pre_order,
    branch_gradients, log_likelihood, lnl_and_grad, postorder_nodes,
)
from .rate_gradient import rate_matrix_gradient

__all__ = [
    "transition_matrices", "tip_partials", "post_order", "root_site_loglik", "pre_order",
    "branch_gradients", "log_likelihood", "lnl_and_grad", "postorder_nodes",
    "rate_matrix_gradient",
]
