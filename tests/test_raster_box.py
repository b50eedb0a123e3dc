"""The rasterizer skips, per 8x8 sub-tile, records whose cutoff box misses
the sub-tile.  The skip must never remove a pixel that the binary32 blend test
(-power <= cutoff) would keep; this checks the box's rounding margin on
ill-conditioned conics by evaluating the power as the kernel does (binary32,
fused multiply-adds emulated by one rounding of the exact FP64 value)."""

import numpy as np

f32 = np.float32
CUTOFF = f32(4.5)
U = 5.9604645e-8


def fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def power32(u, v, A, B, C, px, py):
    dx = (u - px).astype(f32)
    dy = (v - py).astype(f32)
    inner = fma32((A * dx).astype(f32), dx, (C * dy * dy).astype(f32))
    return fma32(np.full_like(inner, f32(-0.5)), inner, (-B * dx * dy).astype(f32))


def box32(u, v, A, B, C):
    det = (A * C - B * B).astype(f32)
    tr = (A + C).astype(f32)
    kap = (tr * tr / det).astype(f32)
    ok = (det > 0) & (kap < f32(1.0e5))
    grow = (f32(2.0) * CUTOFF * (f32(1.002) + f32(64.0) * f32(U) * kap) / det).astype(f32)
    hx = (np.sqrt(grow * C) + f32(0.01)).astype(f32)
    hy = (np.sqrt(grow * A) + f32(0.01)).astype(f32)
    return ok, u - hx, u + hx, v - hy, v + hy


def test_cutoff_box_is_conservative():
    rng = np.random.default_rng(7)
    n = 4000
    # conics of covariances with eigenvalues from 0.3 px^2 (the dilation) to
    # 1e5 px^2 at random orientations, centred anywhere in a 1080p frame
    l1 = 0.3 + rng.uniform(0, 1, n) * 3
    l2 = l1 * 10 ** rng.uniform(0, 4.5, n)
    th = rng.uniform(0, np.pi, n)
    c, s = np.cos(th), np.sin(th)
    sxx = c * c * l1 + s * s * l2
    syy = s * s * l1 + c * c * l2
    sxy = c * s * (l1 - l2)
    det = sxx * syy - sxy * sxy
    A = (syy / det).astype(f32)
    B = (-sxy / det).astype(f32)
    C = (sxx / det).astype(f32)
    u = rng.uniform(0, 1920, n).astype(f32)
    v = rng.uniform(0, 1080, n).astype(f32)
    ok, x0, x1, y0, y1 = box32(u, v, A, B, C)
    checked = 0
    for i in np.nonzero(ok)[0][:600]:
        # every integer pixel in a window beyond the box on all sides
        ax = int(np.floor(x0[i])) - 3, int(np.ceil(x1[i])) + 3
        ay = int(np.floor(y0[i])) - 3, int(np.ceil(y1[i])) + 3
        if (ax[1] - ax[0]) * (ay[1] - ay[0]) > 400_000:
            continue
        ys, xs = np.mgrid[ay[0]:ay[1], ax[0]:ax[1]]
        xs = xs.ravel().astype(f32)
        ys = ys.ravel().astype(f32)
        pw = power32(np.full_like(xs, u[i]), np.full_like(xs, v[i]), np.full_like(xs, A[i]),
                     np.full_like(xs, B[i]), np.full_like(xs, C[i]), xs, ys)
        keep = ~(-pw > CUTOFF)
        inside = (xs >= x0[i]) & (xs <= x1[i]) & (ys >= y0[i]) & (ys <= y1[i])
        assert not np.any(keep & ~inside), i
        checked += 1
    assert checked > 300
    # the box is also tight: its half-width stays within a few percent of
    # the exact extent for well-conditioned conics
    exact_hx = np.sqrt(2 * 4.5 * C.astype(np.float64) / (A.astype(np.float64) * C - B.astype(np.float64) ** 2))
    well = ok & ((A + C) ** 2 / (A * C - B * B) < 100)
    assert np.all((x1 - u)[well] <= exact_hx[well] * 1.01 + 0.02)


def square_may_hit32(u, v, A, B, C, o, x0, y0, ext, alpha_min):
    """The rasterizers' per-wave record test, step by step in binary32 (no
    fused operations, as the kernels are built)."""
    one = f32(1.0)
    dxl, dxh = (u - (x0 + ext)).astype(f32), (u - x0).astype(f32)
    dyl, dyh = (v - (y0 + ext)).astype(f32), (v - y0).astype(f32)
    inside = (dxl <= 0) & (dxh >= 0) & (dyl <= 0) & (dyh >= 0)
    rho = (np.abs(B) * (one / np.sqrt((A * C).astype(np.float64))).astype(f32)).astype(f32)

    def edge(dx, lo, hi, A_, B_, C_):
        rC = (one / C_).astype(f32)  # the kernels take a hardware reciprocal
        dy = np.minimum(np.maximum(((-B_ * dx).astype(f32) * rC).astype(f32), lo), hi)
        return (((A_ * dx).astype(f32) * dx).astype(f32) + ((f32(2.0) * B_ * dx).astype(f32) * dy).astype(f32)
                + ((C_ * dy).astype(f32) * dy).astype(f32)).astype(f32)

    # the edges facing the centre (the x-edge on its side, the y-edge likewise)
    dxe = np.where(dxl > 0, dxl, dxh)
    dye = np.where(dyl > 0, dyl, dyh)
    q = np.minimum(edge(dxe, dyl, dyh, A, B, C), edge(dye, dxl, dxh, C, B, A))
    qlo = (q * (one - (f32(3.8148e-6) * (one / (one - rho)).astype(f32)).astype(f32))).astype(f32)
    pmax = (f32(-0.5) * qlo).astype(f32)
    alpha_ok = (o * np.exp(pmax.astype(np.float64)).astype(f32) * f32(1.0000153)).astype(f32) >= alpha_min
    out = np.where(-pmax > CUTOFF, False, alpha_ok)
    out = np.where((A > 0) & (C > 0) & (rho <= f32(0.999)), out, True)
    return np.where(inside, (o * f32(1.0000153)).astype(f32) >= alpha_min, out)


def test_square_test_is_conservative():
    """The per-wave test never drops a record that some pixel of the wave's
    square takes: every skip is checked against the binary32 power and alpha
    of each of its pixels, for conics from round to 1e4:1 at any orientation,
    opacities down to alpha_min, and squares placed around the cut ellipse."""
    rng = np.random.default_rng(11)
    alpha_min = f32(1.0 / 255.0)
    skipped = checked = 0
    for ext in (7, 3):
        n = 20000
        l1 = 0.3 + rng.uniform(0, 1, n) * 3
        l2 = l1 * 10 ** rng.uniform(0, 4.0, n)
        th = rng.uniform(0, np.pi, n)
        c, s = np.cos(th), np.sin(th)
        sxx = c * c * l1 + s * s * l2
        syy = s * s * l1 + c * c * l2
        sxy = c * s * (l1 - l2)
        det = sxx * syy - sxy * sxy
        A = (syy / det).astype(f32)
        B = (-sxy / det).astype(f32)
        C = (sxx / det).astype(f32)
        o = (10 ** rng.uniform(np.log10(1 / 255), 0, n)).astype(f32)
        # square origin at a pixel; the centre within 1.2x the cut radius of it
        x0 = rng.integers(0, 1900, n).astype(f32)
        y0 = rng.integers(0, 1060, n).astype(f32)
        r = np.sqrt(2 * 4.5 * l2) * 1.2 + ext
        u = (x0 + rng.uniform(-r, r + ext)).astype(f32)
        v = (y0 + rng.uniform(-r, r + ext)).astype(f32)
        may = square_may_hit32(u, v, A, B, C, o, x0, y0, f32(ext), alpha_min)
        # every pixel of every square
        oy, ox = np.mgrid[0:ext + 1, 0:ext + 1]
        px = (x0[:, None] + ox.ravel()[None, :]).astype(f32)
        py = (y0[:, None] + oy.ravel()[None, :]).astype(f32)
        bc = lambda z: np.broadcast_to(z[:, None], px.shape).astype(f32)
        pw = power32(bc(u), bc(v), bc(A), bc(B), bc(C), px, py)
        alpha = np.minimum(f32(0.99), (bc(o) * np.exp(pw.astype(np.float64)).astype(f32)).astype(f32))
        hit = ~(-pw > CUTOFF) & ~(alpha < alpha_min)
        assert not np.any(hit[~may].any(axis=1)), ext
        skipped += int((~may).sum())
        checked += n
        # and it is useful: most squares that no pixel takes are skipped
        none = ~hit.any(axis=1)
        assert (~may).sum() >= 0.8 * none.sum()
    assert skipped > 10000
