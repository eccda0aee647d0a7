"""The GPU spectra (lbm_spectra: moments kernel, FFT, shell sums over the
stored half plane with atomic adds) against the oracle's full-plane
definition, on the moments of the same populations."""
import sys

import numpy as np
import pytest
import torch

from paper_1507_02509_amd import inputs
from paper_1507_02509_amd.sim import Sim, beta_from_nu

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,form", [(64, "f64"), (256, "f64"), (255, "f64"), (256, "f32")])
def test_spectra_match_oracle(orc, n, form):
    """Odd N checks the half-plane weights (no Nyquist column).  Bar: 1e-12
    of the largest shell (FP64 sums in a different order); FP32 storage
    changes only the populations, which both sides read from the GPU."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("spectra", n, form)
    ux, uy = inputs.spectral(n, 8, 0.05, seed=7)
    s = Sim(n, n, beta_from_nu(1e-4), variant="B", form=form).init(ux, uy)
    s.step(20)
    kmax = int(np.ceil(n / np.sqrt(2)))
    ek, zk = (t.cpu().numpy() for t in s.spectra(kmax))
    _, gx, gy = (t.cpu().numpy() for t in s.moments())
    oe, oz = orc.spectra(gx, gy, kmax)
    eE = np.abs(ek - oe).max() / oe.max()
    eZ = np.abs(zk - oz).max() / oz.max()
    say("  E err", eE, "Z err", eZ, "sum E", ek.sum(), "E", 0.5 * np.mean(gx ** 2 + gy ** 2))
    assert eE < 1e-12 and eZ < 1e-12
    assert abs(ek.sum() - 0.5 * np.mean(gx ** 2 + gy ** 2)) < 1e-12 * ek.sum()
    small_e, _ = s.spectra(4)
    assert np.abs(small_e.cpu().numpy() - oe[:5]).max() < 1e-12 * oe.max()


def test_spectra_reject_non_square():
    from paper_1507_02509_amd import _lib as L
    s = Sim(64, 32, beta_from_nu(1e-3), variant="B", form="f32").init(np.zeros((32, 64)), np.zeros((32, 64)))
    with pytest.raises(L.KbcError):
        s.spectra(8)
