"""Host logic of the warm start: a predicted shock profile is moved along the
line so that its density crosses the mean of the two states at L/2 (where the
cold start puts its shock), keeping its shape and extending its plateaus; the
network's normalised outputs become the moment fields of the two jump states."""
import numpy as np

from paper_2201_05280_amd import cases as C
from paper_2201_05280_amd.inputs import positions
from paper_2201_05280_amd.shock import profile_metrics


def _profile(L, centre, width=3.0):
    x = positions(L, 1, 1)[0]
    f = 0.5 * (1 + np.tanh((x - centre) / width))
    return np.stack([f, f ** 2, np.sqrt(f), 1 - (1 - f) ** 2], 1)


def test_recentred_shock_crosses_the_mean_at_half_length():
    L = 300
    x = positions(L, 1, 1)[0]
    for centre in (150.0, 171.3, 120.6):
        ys = _profile(L, centre)
        r = C.recentre_shock(L, ys)
        pos, thick = profile_metrics(x, r[:, 0], (0.0, 0, 0), (1.0, 0, 0))
        pos0, thick0 = profile_metrics(x, ys[:, 0], (0.0, 0, 0), (1.0, 0, 0))
        # crossings are located by linear interpolation between sites half a
        # cell apart: exact up to the profile's curvature there
        assert abs(pos0 - centre) < 5e-3
        assert abs(pos - L / 2) < 5e-3
        assert abs(thick - thick0) < 3e-2 * thick0   # the shape is kept (linear re-sampling)
        # every output moves by the same shift, and the plateaus extend
        shift = centre - L / 2
        inner = np.abs(x - L / 2) < L / 2 - abs(shift) - 20
        ref = _profile(L, L / 2)
        assert np.abs(r[inner] - ref[inner]).max() < 1e-2   # linear re-sampling error
        assert r[np.argmin(x)].max() < 1e-12 + ys[np.argmin(x)].max()
        assert np.allclose(r[np.argmax(x)], 1.0, atol=1e-9)


def test_profile_without_a_crossing_is_left_as_predicted():
    L = 64
    ys = np.full((2 * L, 4), 0.3)
    assert np.array_equal(C.recentre_shock(L, ys), ys)


def test_prediction_maps_onto_the_jump_states():
    L = 40
    case = dict(kind=C.SHOCK, L=L, U=1.0, up=(1.0, 0.9, 0.3), down=(1.8, 0.5, 0.4))
    ys = _profile(L, 25.0)
    f = C.fields_from_prediction([case], ys, recentre_shocks=True)
    x = positions(L, 1, 1)[0]
    pos, _ = profile_metrics(x, f["rho"], case["up"], case["down"])
    assert abs(pos - L / 2) < 5e-3
    assert f["rho"].min() >= 1.0 - 1e-12 and f["rho"].max() <= 1.8 + 1e-12
    assert np.allclose(f["u"][1:], 0.0)
