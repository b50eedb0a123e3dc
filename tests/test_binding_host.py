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


def test_sort_mode_choice():
    """'tiles' and 'global' are taken as given; 'auto' (the default) takes the
    per-tile sort only once a capacity fit has seen every list shorter than
    TILE_SORT_MAX entries, and set_flags forgets that measurement."""
    from paper_2503_08217_amd import _abi as A
    from paper_2503_08217_amd.renderer import TILE_SORT_MAX, Renderer
    c = scenes.make_config(1)
    tiles = lambda r: bool(r.c_params.flags & A.S3R_SORT_TILES)  # noqa: E731
    assert tiles(Renderer(c.scene, c.views, dict(c.params, sort="tiles"), device="cpu"))
    assert not tiles(Renderer(c.scene, c.views, dict(c.params, sort="global"), device="cpu"))
    r = Renderer(c.scene, c.views, dict(c.params), device="cpu")
    assert not tiles(r)  # nothing measured yet
    r._max_list = TILE_SORT_MAX - 1
    r.c_params = r.make_params()
    assert tiles(r)
    r._max_list = TILE_SORT_MAX
    r.c_params = r.make_params()
    assert not tiles(r)
    r._max_list = 10
    r.set_flags(lod=True)
    assert r._max_list is None and not tiles(r)
    with pytest.raises(ValueError):
        Renderer(c.scene, c.views, dict(c.params, sort="bogus"), device="cpu")
