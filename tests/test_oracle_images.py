"""Pins of the oracle's image projections (Sec. 2.6.1 binned images, Sec. 2.6.2
peeled images), from closed forms on an empty grid.

On an empty grid a packet flies straight from its source to the boundary, so
its escape point is x_s + t d.  The binned image projects that point on the
plane perpendicular to d, with e_x = norm(z x d) and e_y = d x e_x; the t d
part drops out, and for a source on the z axis at height z_s the projection is
exactly (X, Y) = (0, z_s sin(theta)), theta the angle of d from the z axis.
With isotropic emission |mu| = |d_z| is uniform on [0, 1], so the share of an
inclination bin's packets that lands in a pixel row follows from the row's
band of sin(theta) in closed form.  For a source on the x axis at x_s,
X = -x_s sin(phi), phi uniform, which fixes the share per pixel column.

A peeled image collects, on an empty grid, only the direct peel of each
emission: every packet adds eps/(4 pi) at the source position projected along
the observer direction o.  The axes of the listed observers are worked out by
hand below (e_x = norm(z x o), or x when o is the z axis; e_y = o x e_x), so
the whole image sits in one pixel that is known in advance.

Each test fails on a swapped image axis, a sign flip of e_y, a missing
normalisation of e_x or a transposed pixel index.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1112_1071_amd import synth

AU = synth.AU


def _empty_model(src_pos, npix, n_packets, k_img=7, n_bins=20, peel_dirs=None):
    cfg = synth.config0(n=16, n_packets=n_packets, n_iter=1, n_bins=n_bins)
    cfg["rho"][:] = 0.0
    spec = np.zeros(n_bins)
    spec[k_img] = 1.0  # every packet in the image bin
    cfg["sources"] = [{"pos": list(src_pos), "lum": synth.L_SUN, "spectrum": spec}]
    cfg["observers"] = {"n_incl": 10, "img_npix": npix, "img_half_width": 1.0 * AU,
                        "img_nu_bins": [k_img]}
    if peel_dirs is not None:
        cfg["peeloff"] = {"dirs": peel_dirs}
    return cfg


def _band_share(lo, hi, a, b):
    """length of [lo, hi) intersected with [a, b)"""
    return max(0.0, min(hi, b) - max(lo, a))


def test_binned_image_of_a_source_on_the_z_axis(orc):
    npix, n_packets, zs = 33, 400_000, 0.53
    cfg = _empty_model([0.0, 0.0, zs * AU], npix, n_packets)
    m = oracle.OracleModel(cfg)
    m.final_pass()
    img, _ = m.images()
    sed, _, cnt = m.sed()
    eps = synth.L_SUN / n_packets
    # every escape lands in the central column (X = 0 is the middle of pixel 16)
    col = img[0].sum(axis=1)  # [incl][x]
    assert col[:, 16].sum() == pytest.approx(synth.L_SUN, rel=1e-12)
    assert not np.any(np.delete(col, 16, axis=1))
    # rows: Y = zs sin(theta) > 0, so only rows at or above the centre
    width = 2.0 / npix  # pixel width in AU
    for i in range(10):
        rows = img[0, i, :, 16] / eps
        assert rows.sum() == pytest.approx(cnt[i, 7], abs=0.5)
        a, b = i / 10, (i + 1) / 10  # |mu| band of the inclination bin
        n_i = 0
        for r in range(npix):
            y0, y1 = -1.0 + r * width, -1.0 + (r + 1) * width
            # sin(theta) in [y0/zs, y1/zs)  <=>  |mu| in (sqrt(1-(y1/zs)^2), sqrt(1-(y0/zs)^2)]
            s0, s1 = max(y0 / zs, 0.0), min(y1 / zs, 1.0)
            p = 0.0
            if s1 > s0:
                p = _band_share(math.sqrt(1 - s1 * s1), math.sqrt(1 - s0 * s0), a, b)
            expect = n_packets * p
            if p == 0.0:
                assert rows[r] == 0, (i, r, rows[r])
            else:
                z = (rows[r] - expect) / math.sqrt(expect * (1 - p))
                assert abs(z) < 4.5, (i, r, rows[r], expect)
                n_i += 1
        assert n_i >= 1
    # the rows at and below the centre line (Y <= 0) stay empty
    assert not np.any(img[0, :, : npix // 2, :])


def test_binned_image_columns_of_a_source_on_the_x_axis(orc):
    # X = -xs sin(phi), phi uniform: P(X in [x0, x1)) = (asin(-x0/xs) - asin(-x1/xs)) / pi
    npix, n_packets, xs = 20, 400_000, 0.47
    cfg = _empty_model([xs * AU, 0.0, 0.0], npix, n_packets)
    m = oracle.OracleModel(cfg)
    m.final_pass()
    img, _ = m.images()
    eps = synth.L_SUN / n_packets
    cols = img[0].sum(axis=(0, 1)) / eps  # all inclinations
    width = 2.0 / npix
    for c in range(npix):
        x0, x1 = -1.0 + c * width, -1.0 + (c + 1) * width
        u0, u1 = max(-x1 / xs, -1.0), min(-x0 / xs, 1.0)
        p = (math.asin(u1) - math.asin(u0)) / math.pi if u1 > u0 else 0.0
        if p == 0.0:
            assert cols[c] == 0, (c, cols[c])
        else:
            z = (cols[c] - n_packets * p) / math.sqrt(n_packets * p * (1 - p))
            assert abs(z) < 4.5, (c, cols[c], n_packets * p)


# Observer directions with their image axes worked out by hand:
# o, e_x = norm(z x o) (x for the z axis), e_y = o x e_x.
HAND_AXES = [
    ([0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]),
    ([1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]),
    ([0.6, 0.0, 0.8], [0.0, 1.0, 0.0], [-0.8, 0.0, 0.6]),
    ([0.0, -0.28, -0.96], [1.0, 0.0, 0.0], [0.0, -0.96, 0.28]),
    ([0.0, 0.6, 0.8], [-1.0, 0.0, 0.0], [0.0, -0.8, 0.6]),
]


def test_peeled_image_pixel_of_the_source(orc):
    npix, n_packets = 20, 4000
    src = np.array([0.33, -0.47, 0.58])  # AU
    dirs = [o for o, _, _ in HAND_AXES]
    cfg = _empty_model(list(src * AU), npix, n_packets, peel_dirs=dirs)
    m = oracle.OracleModel(cfg)
    m.final_pass()
    img, _ = m.peeled_images()
    psed, _ = m.peeled_sed()
    width = 2.0 / npix
    for i, (o, ex, ey) in enumerate(HAND_AXES):
        X, Y = float(np.dot(src, ex)), float(np.dot(src, ey))
        fx, fy = (X + 1.0) / width, (Y + 1.0) / width
        # the test point sits well inside its pixel
        assert min(fx % 1, 1 - fx % 1, fy % 1, 1 - fy % 1) > 0.1
        want = np.zeros((npix, npix))
        want[int(fy), int(fx)] = synth.L_SUN / (4 * math.pi)
        np.testing.assert_allclose(img[0, i], want, rtol=1e-12, atol=0.0)
        assert psed[i, 0, 7] == pytest.approx(synth.L_SUN / (4 * math.pi), rel=1e-12)
