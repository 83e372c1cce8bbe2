"""GPU test of the accuracy-study driver (Sec. 3.1): on a reduced tube, the
error of the velocity profile saturates at a small population count in the
near-hydrodynamic regime (about 100 populations at Kn = 0.05) and keeps
falling with the population count in the near-ballistic one (Kn = 10), the
behaviour Sec. 3.1 reports for its Fig. 3."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_tube_error_depends_on_angles_only_beyond_hydro():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import studies
    log = lambda m: print(m, file=sys.stderr, flush=True)
    res = studies.tube_study(Kns=(0.05, 10.0), Ks=(8, 24, 96), L=400, refine=2, K_ref=240, log=log)
    lo, hi = res[0.05]["eps"], res[10.0]["eps"]
    log("Kn 0.05: %s  Kn 10: %s" % (lo, hi))
    # N_pop = 32, 96, 384
    assert lo[1] < 1.2 * lo[2]                               # Kn 0.05: saturated by N_pop ~ 100
    assert res[0.05]["saturation_npop"] <= 96
    assert hi[0] > hi[1] > 2 * hi[2]                         # Kn 10: still falling beyond 96


def test_tube_study_numbers_match_the_oracle():
    """The study's error numbers on the GPU path equal those of the same runs
    on the FP64 oracle (the runs agree to rounding, so the errors do too)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import studies
    from test_oracle_studies import oracle_tube_errors
    log = lambda m: print(m, file=sys.stderr, flush=True)
    Ks = (8, 24, 96)
    res = studies.tube_study(Kns=(0.05, 10.0), Ks=Ks, L=200, refine=2, K_ref=120, log=log)
    for Kn in (0.05, 10.0):
        ref = oracle_tube_errors(200, 2, 120, Ks, Kn)
        log("Kn %g: GPU %s oracle %s" % (Kn, res[Kn]["eps"], ref))
        np.testing.assert_allclose(res[Kn]["eps"], ref, rtol=1e-9)
