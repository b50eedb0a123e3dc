"""Host side of the binding, without a GPU: buffers are allocated (on the
CPU device) and marshalled into the C structs for every option combination;
no kernel is launched."""

import pytest

import scenes

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("extra", [{}, {"raster_mask": True, "grad_sparse": True},
                                   {"lod_stochastic": True, "tile": 32}])
def test_renderer_marshals_on_host(plain, extra):
    from paper_2503_08217_amd import _abi as A
    from paper_2503_08217_amd.renderer import Renderer
    c = scenes.make_config(1)
    r = Renderer(c.scene, c.views, dict(c.params, **extra), device="cpu", plain=plain)
    assert r.c_img.n == c.scene.n
    assert bool(r.c_img.m_raster) == bool(extra.get("raster_mask"))
    assert bool(r.c_grads.rows) and bool(r.c_proj.surv) and bool(r.c_bins.tile_order)
    f = r.c_params.flags
    assert bool(f & A.S3R_PLAIN) == plain
    assert bool(f & A.S3R_GRAD_SPARSE) == bool(extra.get("grad_sparse"))
    assert bool(f & A.S3R_LOD_STOCHASTIC) == bool(extra.get("lod_stochastic"))
    assert r.c_params.tile == extra.get("tile", 16)
    # every view batch prepared later must fit the buffers of the first
    with pytest.raises(ValueError):
        r.prepare_views([scenes.make_config(2, scale_n=0.001).views.subset([0, 1, 2, 3])])
