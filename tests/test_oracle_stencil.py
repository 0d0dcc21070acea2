"""Pins of the oracle's sampling stencil (CPU only): the image Jacobian in closed form and the
exact set of valid correspondences.

Image Jacobians (Supplementary): the GN-mode Jacobian of a channel at u' = (u, v) is the
bilinear blend of the central differences 1/2 (I[x+1] - I[x-1]) (columns) and
1/2 (I[y+1] - I[y-1]) (rows) taken at the four bilinear taps.  On a quadratic texture
I = alpha x^2 + beta y^2 + gamma x y + c0 (x = column, y = row) those differences are exact:
2 alpha x + gamma y and 2 beta y + gamma x, linear in the tap position, so their bilinear blend is
that linear function at u':  G = (2 alpha u + gamma v, 2 beta v + gamma u).  The slope of the
bilinear interpolant (exact-derivative mode) is instead G = (alpha (2 x0 + 1) + gamma v,
beta (2 y0 + 1) + gamma u) for the cell (x0, y0).  With dyadic coefficients every texel is exact in
FP32, so both forms hold to FP64 rounding at every valid pixel and for every channel; a wrong tap
row or column, or blend weights attached to the wrong taps, moves G by O(alpha).

Border rule (reading of the paper's silence on borders): the cell is floor(u') and all 12 taps of
the stencil must lie inside the image, 1 <= floor(u) <= W - 3 and 1 <= floor(v) <= H - 3.  A
fronto-parallel plane seen again by a camera moved parallel to it by (kx, ky) pixels' worth maps
every pixel (c, r) to u' = (c - kx, r - ky); with half-pixel fractions no decision is near a
tie, so the valid set is known pixel by pixel in closed form.
"""
import numpy as np
import pytest

import oracle
import synth

# (alpha, beta, gamma, c0) per channel: intensity, depth, normal x, y, z (all dyadic)
QUAD = [
    (2.0 ** -16, 2.0 ** -15, 2.0 ** -17, 0.25),
    (2.0 ** -15, -(2.0 ** -16), 2.0 ** -14, 3.0),
    (-(2.0 ** -17), 2.0 ** -16, 2.0 ** -15, 0.125),
    (2.0 ** -14, 2.0 ** -17, -(2.0 ** -16), -0.5),
    (2.0 ** -16, -(2.0 ** -14), 2.0 ** -17, -0.75),
]


def quadratic_images(H, W):
    """The five quadratic channel images (FP64 values, exactly representable in FP32)."""
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    imgs = [al * x * x + be * y * y + ga * x * y + c0 for (al, be, ga, c0) in QUAD]
    for im in imgs:
        assert np.array_equal(im.astype(np.float32).astype(np.float64), im)
    return imgs


def with_quadratic_target(p, t):
    """A copy of problem p whose keyframe t carries the quadratic channels."""
    H, W = p.depth[t].shape
    I, D, nx, ny, nz = quadratic_images(H, W)
    q = synth.Problem(p.name + "_quad", p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs, dict(p.params))
    q.intensity, q.depth, q.normals = list(p.intensity), list(p.depth), list(p.normals)
    q.intensity[t] = I.astype(np.float32)
    q.depth[t] = D.astype(np.float32)
    q.normals[t] = np.stack([nx, ny, nz], -1).astype(np.float32)
    return q


def closed_form_G(uv, grad_mode):
    """Expected [N, 5, 2] image Jacobians at projected points uv [N, 2]."""
    u, v = uv[:, 0], uv[:, 1]
    x0, y0 = np.floor(u), np.floor(v)
    out = np.empty((len(u), 5, 2))
    for ch, (al, be, ga, _) in enumerate(QUAD):
        if grad_mode == 0:
            out[:, ch, 0] = 2 * al * u + ga * v
            out[:, ch, 1] = 2 * be * v + ga * u
        else:
            out[:, ch, 0] = al * (2 * x0 + 1) + ga * v
            out[:, ch, 1] = be * (2 * y0 + 1) + ga * u
    return out


def quadratic_G_error(p, s, t, grad_mode):
    """max |G_oracle - G_closed_form| over the valid pixels of pair (s, t) with a quadratic target
    (occlusion gate and Huber disabled), the number of valid pixels, and the largest error of
    the bilinear intensity value V = I_s - e_I against its closed form."""
    q = with_quadratic_target(p, t)
    prm = dict(q.params, channels=5, occ_tau_pinhole=1e9, occ_tau_spherical=1e9, huber_delta=1e9)
    r = oracle.eval_pair(q, q.init_poses, s, t, prm, pixels=True, grad_mode=grad_mode)
    v = r["status"] == oracle.ST_VALID
    uv = r["uv"][v]
    G = r["G"][v]
    err = np.abs(G - closed_form_G(uv, grad_mode)).max() if v.any() else np.inf
    # value: the bilinear interpolant of x^2 is x0^2 + a (2 x0 + 1); of x y it is x y exactly
    al, be, ga, c0 = QUAD[0]
    x0, y0 = np.floor(uv[:, 0]), np.floor(uv[:, 1])
    a, b = uv[:, 0] - x0, uv[:, 1] - y0
    Vexp = al * (x0 * x0 + a * (2 * x0 + 1)) + be * (y0 * y0 + b * (2 * y0 + 1)) + ga * uv[:, 0] * uv[:, 1] + c0
    Vorc = q.intensity[s].astype(np.float64)[v] - r["res"][v][:, 0]
    verr = np.abs(Vorc - Vexp).max() if v.any() else np.inf
    return err, int(v.sum()), verr, uv


@pytest.mark.parametrize("fixture", ["rgbd_small", "lidar_mini"])
@pytest.mark.parametrize("grad_mode", [0, 1])
def test_image_jacobian_closed_form_on_quadratic_textures(fixture, grad_mode, request):
    """Pinhole and spherical targets: the per-pixel image Jacobian of every channel equals its
    closed form to 1e-12 at every valid pixel, and the bilinear value its closed form; the pixels
    cover the whole range of sub-pixel fractions in both directions."""
    p = request.getfixturevalue(fixture)
    err, n, verr, uv = quadratic_G_error(p, 1, 0, grad_mode)
    assert n > 2000
    assert err < 1e-12, err
    assert verr < 1e-12, verr
    frac = uv - np.floor(uv)
    for k in range(2):
        h, _ = np.histogram(frac[:, k], bins=4, range=(0, 1))
        assert h.min() > n / 20   # fractions spread over [0, 1) in both directions


# ---------------------------------------------------------------- border rule: exact valid set

def shifted_plane_problem(kx, ky, Z=3.0, holes=()):
    """Two keyframes of the 160 x 120 pinhole camera (fx = fy = 120) facing a plane at depth Z;
    the second camera is moved by (kx Z / fx, ky Z / fy, 0), so source pixel (c, r) lands at
    u' = (c - kx, r - ky).  `holes`: target pixels (col, row) without a depth measurement."""
    p = synth.make("rgbd_small", render_images=False)
    sen = p.sensors[0]
    H, W = sen["H"], sen["W"]
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    I = (0.5 + 0.25 * np.sin(0.3 * x) * np.cos(0.2 * y)).astype(np.float32)
    D = np.full((H, W), Z, np.float32)
    Dt = D.copy()
    for (c, r) in holes:
        Dt[r, c] = 0.0
    Nn = np.zeros((H, W, 3), np.float32)
    Nn[..., 2] = -1.0
    p.intensity, p.depth, p.normals = [I, I], [D, Dt], [Nn, Nn]
    p.kf_sensor = np.zeros(2, np.int32)
    eye = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float64)
    X1 = eye.copy()
    X1[9] = kx * Z / sen["fx"]
    X1[10] = ky * Z / sen["fy"]
    return p, np.stack([eye, X1]), H, W


def expected_valid(kx, ky, H, W, holes=()):
    """Source pixels whose cell floor(c - kx), floor(r - ky) keeps the 12-tap stencil inside the
    image and whose stencil (the 2x2 bilinear taps and their 4-neighbours) avoids every hole."""
    r, c = np.mgrid[0:H, 0:W]
    x0 = np.floor(c - kx).astype(int)
    y0 = np.floor(r - ky).astype(int)
    ok = (x0 >= 1) & (x0 <= W - 3) & (y0 >= 1) & (y0 <= H - 3)
    for (hc, hr) in holes:
        hit = np.zeros_like(ok)
        for (dx, dy) in ((0, 0), (1, 0), (0, 1), (1, 1)):
            tx, ty = x0 + dx, y0 + dy
            for (ex, ey) in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
                hit |= (tx + ex == hc) & (ty + ey == hr)
        ok &= ~hit
    return ok


def valid_set(kx, ky, holes=()):
    p, X, H, W = shifted_plane_problem(kx, ky, holes=holes)
    r = oracle.eval_pair(p, X, 0, 1, dict(p.params, channels=5), pixels=True)
    return r, H, W


@pytest.mark.parametrize("kx,ky", [(2.5, 0.5), (-2.5, 0.5), (2.5, -0.5), (-2.5, -0.5)])
def test_border_rule_exact_valid_set(kx, ky):
    """Every source pixel is valid exactly when 1 <= floor(u') <= W - 3 and 1 <= floor(v') <= H - 3:
    (W - 4) x (H - 3) pixels for a half-pixel shift of 2.5 columns and 0.5 rows in either
    direction, at the exact positions, with the sub-pixel fractions 1/2."""
    r, H, W = valid_set(kx, ky)
    v = r["status"] == oracle.ST_VALID
    exp = expected_valid(kx, ky, H, W)
    assert exp.sum() == (W - 4) * (H - 3)
    np.testing.assert_array_equal(v, exp)
    np.testing.assert_allclose(r["uv"][v] - np.floor(r["uv"][v]), 0.5, atol=1e-9)


def test_missing_depth_tap_removes_exactly_the_stencils_that_read_it():
    """A target texel without depth invalidates exactly the 12 cells whose stencil contains it
    (4x4 block minus its corners): 12 source pixels for an interior hole, none elsewhere."""
    kx, ky = 2.5, 0.5
    holes = [(70, 50), (120, 33)]
    r, H, W = valid_set(kx, ky, holes=holes)
    v = r["status"] == oracle.ST_VALID
    base = expected_valid(kx, ky, H, W)
    exp = expected_valid(kx, ky, H, W, holes=holes)
    assert base.sum() - exp.sum() == 24
    np.testing.assert_array_equal(v, exp)
    assert np.all(r["status"][base & ~exp] == oracle.ST_BADTAP)
