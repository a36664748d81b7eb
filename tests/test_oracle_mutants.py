"""The oracle's pins have power: each plausible mistake planted in the oracle
(a compile-time switch, built only here, on the CPU) makes its pin fail."""
import pytest

from tests import test_oracle_mlp as M
from tests import test_oracle_pins as P
from tests import test_oracle_shift as S
from tests import test_oracle_events as E
from tests import test_oracle_exact as X
from tests import test_oracle_three_level as T

MUTANTS = [
    # (switch, what is wrong, the pin that must fail)
    (1, "nu density as printed: nu/gamma_g in the sum", lambda o: P.test_nu_conditional(o)),
    (2, "gamma shape nu/2 + N instead of nu/2 + N/2", lambda o: P.test_gamma_conditional(o)),
    (3, "sigma^2 shape G/2: the Jacobian of the U(0, s) prior on sigma dropped",
     lambda o: P.test_sigma2_conditional(o, 100.0, 6)),
    (4, "slice window not placed at random around x0",
     lambda o: P.test_slice_step_is_stationary(o, *P.TARGETS[0])),
    (5, "beta sufficient statistic taken from the wrong design column",
     lambda o: P.test_beta_conditional(o, "cell_means")),
    (6, "eps likelihood with exp(eta - eps)", lambda o: P.test_eps_conditional(o)),
    (7, "theta drawn with sd 1/precision instead of 1/sqrt(precision)",
     lambda o: P.test_theta_conditional(o)),
    (8, "tau rate b + nu sum 1/gamma instead of b + (nu/2) sum 1/gamma",
     lambda o: P.test_tau_conditional(o)),
    (9, "independence MH acceptance without the proposal-density ratio",
     lambda o: M.test_imh_step_is_stationary(o, "cell_means", *M.PROPOSALS[1])),
    (10, "shift step moves eps by +X delta instead of -X delta",
     lambda o: S.test_shift_keeps_the_likelihood_sums(o, "paper")),
    (11, "shift step mean without the prior term (beta - theta) / sigma^2",
     lambda o: S.test_shift_draws_the_conditional(o, "two_group")),
    (12, "contrast event as 'any row' instead of 'all rows'",
     lambda o: E.test_event_counts_match_a_recount(o)),
    (13, "Marsaglia-Tsang constant d = alpha - 1/2 instead of alpha - 1/3",
     lambda o: X.test_exact_gamma_conditional(o)),
    (14, "shape-below-one exponent 1/(alpha + 1) instead of 1/alpha",
     lambda o: X.test_exact_gamma_shape_below_one(o)),
    (15, "exact gamma_g draw with scale nu tau + S/2 instead of nu tau/2 + S/2",
     lambda o: X.test_exact_gamma_conditional(o)),
    (16, "exact sigma^2 draw ignores the truncation at s_l^2",
     lambda o: X.test_exact_sigma2_falls_back_to_slice(o)),
    (17, "top-level psi precision without the prior term 1/c0^2",
     lambda o: T.test_top_psi_conditional(o)),
    (18, "top-level b rate sum tau_k without the prior rate b_b",
     lambda o: T.test_top_b_conditional(o)),
    (19, "group theta mean without the top-level prior mean psi_l",
     lambda o: T.test_group_theta_uses_psi(o)),
]


@pytest.mark.parametrize("k,what,pin", MUTANTS, ids=[f"mutant{m[0]}" for m in MUTANTS])
def test_pin_catches_mutant(oracle_lib, k, what, pin):
    o = oracle_lib.variant(k)
    with pytest.raises(AssertionError):
        pin(o)
