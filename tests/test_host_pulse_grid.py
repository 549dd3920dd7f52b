"""The uniform fine-grid initial data of the learned-tagger evaluation (its
reference run): the Fourier tensor-product DOFs of the Gaussian pulse equal
the directly integrated ones (Gauss-Legendre cell averages, point values of
the periodised Gaussian)."""
import numpy as np
import pytest

import afsynth


@pytest.mark.parametrize("seed", [0, 7])
def test_pulse_grid_dofs_match_quadrature(seed):
    torch = pytest.importorskip("torch")
    from paper_2205_07572_amd.tagger_train import pulse_grid_dofs
    n, alpha = 64, 200.0
    data = afsynth.gaussian_pulse(seed, alpha)
    g = pulse_grid_dofs(data, alpha, n, torch.float64, device="cpu")
    ref = afsynth.dofs_periodic(data, n, n, nq=8)
    for kind in ("avg", "corner", "xedge", "yedge"):
        got = g[kind].numpy()
        assert got.shape == (n, n)
        assert np.abs(got - ref[kind][0]).max() <= 1e-12, kind
