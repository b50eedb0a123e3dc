"""The binary32 decisions agree with the FP64 route away from thresholds."""

import numpy as np
import pytest

import scenes
from oracle import decide32, project64


def _near(a, b, rel):
    return np.abs(a - b) <= rel * np.maximum(np.abs(a), np.abs(b)) + 1e-30


@pytest.mark.parametrize("cfg,v", [(1, 0), (1, 2), (2, 5), (2, 30)])
def test_decisions_match_fp64_outside_guard_band(cfg, v):
    c = scenes.make_config(cfg, scale_n=0.05 if cfg > 1 else 1.0)
    p = dict(c.params)
    args = (c.scene, c.views.W[v], c.views.K[v], c.views.wh[v], int(c.views.tstep[v]), p)
    d32 = decide32.project_cull32(*args)
    d64 = project64.project64(*args)
    # values agree to binary32 accuracy where the Gaussian is in front of the camera
    ok = d64["depth_ok"] & d32["depth_ok"]
    np.testing.assert_allclose(d32["u"][ok], d64["u"][ok], rtol=1e-5, atol=1e-3)
    np.testing.assert_allclose(d32["a_raw"][ok], d64["cov2d"][ok, 0, 0], rtol=2e-3, atol=1e-6)
    # decisions: every mismatch must sit within rounding distance of a threshold
    mism = d32["visible"] != d64["visible"]
    s = p["tile"]
    edge = (_near(d64["pz"], p["z_near"], 1e-5)
            | np.isclose(np.mod(d64["u"] - d64["rad"], s), 0, atol=1e-3)
            | np.isclose(np.mod(d64["u"] + d64["rad"], s), 0, atol=1e-3)
            | np.isclose(np.mod(d64["v"] - d64["rad"], s), 0, atol=1e-3)
            | np.isclose(np.mod(d64["v"] + d64["rad"], s), 0, atol=1e-3)
            | (d32["rad"] != d64["rad"]))
    assert np.all(edge[mism]), np.nonzero(mism & ~edge)
    rad_m = d32["rad"][ok] != d64["rad"][ok]
    x = 3.0 * np.sqrt(d64["lam_d"][ok][rad_m])
    assert np.all(np.abs(x - np.round(x)) < 1e-3)
    assert mism.sum() <= max(2, 1e-4 * c.scene.n)
    ms = d32["surv"] != d64["surv"]
    lod_edge = _near(d64["lam_raw"], p["lod_r"] ** 2, 1e-4)
    assert np.all((edge | lod_edge)[ms])


def test_plain_route_decisions_match_streamlined():
    """The conventional transform in binary32 changes only roundings: the two
    routes decide the same except within rounding distance of a threshold."""
    c = scenes.make_config(2, scale_n=0.05)
    p = scenes.default_params(tile=16)
    for v in (3, 20, 41):
        args = (c.scene, c.views.W[v], c.views.K[v], c.views.wh[v], int(c.views.tstep[v]), p)
        a = decide32.project_cull32(*args)
        b = decide32.project_cull32(*args, plain=True)
        assert (a["visible"] != b["visible"]).sum() <= 2
        np.testing.assert_allclose(a["u"][a["visible"]], b["u"][a["visible"]], rtol=1e-5, atol=2e-3)


@pytest.mark.parametrize("cfg,v", [(1, 1), (2, 17)])
def test_conic_and_colour_match_fp64(cfg, v):
    c = scenes.make_config(cfg, scale_n=0.05 if cfg > 1 else 1.0)
    args = (c.scene, c.views.W[v], c.views.K[v], c.views.wh[v], int(c.views.tstep[v]), c.params)
    d32 = decide32.project_cull32(*args)
    d64 = project64.project64(*args)
    s = d32["surv"] & d64["surv"]
    con32 = np.stack([d32["conic_a"], d32["conic_b"], d32["conic_c"]], 1)[s]
    scale = np.abs(d64["conic"][s]).max(1, keepdims=True)
    np.testing.assert_allclose(con32 / scale, d64["conic"][s] / scale, atol=2e-4)


def test_fp64_autograd_forward_equals_binary32_composite():
    """The torch FP64 forward (conventional route, own projection) reproduces
    the numpy blending of the binary32 projected attributes to binary32 accuracy."""
    from oracle import grad, render
    c = scenes.make_config(1)
    for v in range(3):
        o = render.render_view(c.scene, c.views, v, c.params)
        pt = grad.to_torch_params(c.scene, requires_grad=False)
        img, T = grad.render_t(pt, c.scene, c.views, v, o["order"], c.params)
        ok = ~o["flag"]
        np.testing.assert_allclose(img.numpy()[:, ok], o["image"][:, ok], atol=5e-5)
