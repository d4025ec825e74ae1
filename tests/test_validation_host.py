"""Host-side checks of the total-error estimate (Sec. 4.3) that need no GPU."""
import pytest

import paper_1507_04769_amd as S
from paper_1507_04769_amd import validation as VA


def test_estimator_rejects_empty_reference_mesh():
    # checked on the host, before any plan is made
    with pytest.raises(ValueError):
        VA.Estimator(S.Problem(N=64), 0)


def test_sample_recipe():
    assert VA.N_SAMPLES == 1280  # the paper's sample size


def test_reference_tolerance_and_order():
    # the paper's reference tolerance (1e-7, Sec. 5.1) and the orders of the
    # two reference formulas (checked on the host; plans are not made for the
    # Lobatto reference)
    assert VA.REF_TOL == 1e-7
    with pytest.raises(ValueError):
        VA.Estimator(S.Problem(N=64), 8, scheme=5)
