"""Pins of the CPU oracle against closed forms, brute force and exact special cases.

Every check here comes from outside the oracle: a value derived by hand from the
paper's equations, a brute-force search, an invariant of the mathematics or a
library routine. A plausible slip in the oracle (wrong rounding, wrong border
rule, a dropped term, a flipped sign or a transposed operand) fails at least one.
"""
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synthgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# --------------------------------------------------------------------------
# Pyramid (Sec. III-C, eqs. 1-3)
# --------------------------------------------------------------------------


def _golden_pyramid():
    rows = []
    with open(os.path.join(GOLDEN, "pyramid_closed_forms.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, x, y, v = line.split()[:4]
                rows.append((name, int(x), int(y), int(v)))
    return rows


def _case_image(name):
    img = np.zeros((64, 64), np.uint8)
    if name.startswith("impulse_even"):
        img[32, 32] = 255
    elif name.startswith("impulse_odd"):
        img[32, 33] = 255
    elif name == "tie_half":
        img[34, 34] = 128
    elif name == "border_column":
        img[:, 0] = 255
    return img


@pytest.mark.parametrize("name,x,y,expected", _golden_pyramid())
def test_pyramid_closed_forms(name, x, y, expected):
    lvl1 = oracle.pyramid(_case_image(name), 2)[1]
    assert lvl1[y, x] == expected


def test_pyramid_constant():
    for v in (0, 1, 128, 255):
        for lvl in oracle.pyramid(np.full((75, 97), v, np.uint8), 4):
            assert (lvl == v).all()


def test_pyramid_linear_ramp_is_reproduced():
    # the binomial kernel is symmetric with unit gain, so a linear function
    # a*x + b*y + c maps to a*2x + b*2y + c exactly away from the border
    a, b, c = 1, 2, 7
    yy, xx = np.mgrid[0:60, 0:80]
    img = (a * xx + b * yy + c).astype(np.uint8)
    lvl1 = oracle.pyramid(img, 2)[1]
    Y, X = np.mgrid[0:30, 0:40]
    want = a * 2 * X + b * 2 * Y + c
    assert (lvl1[1:-1, 1:-1] == want[1:-1, 1:-1]).all()


def test_pyramid_sizes():
    lv = oracle.pyramid(np.zeros((135, 135), np.uint8), 3)
    assert [l.shape for l in lv] == [(135, 135), (67, 67), (33, 33)]
    lv = oracle.pyramid(np.zeros((480, 752), np.uint8), 4)
    assert [l.shape for l in lv] == [(480, 752), (240, 376), (120, 188), (60, 94)]


def _direct_eq1(img):
    """Eq. (1) taken literally: one 5x5 weighted sum, one rounding, clamped taps."""
    h, w = img.shape
    wts = np.array([1, 4, 6, 4, 1], np.int64)
    out = np.zeros((h // 2, w // 2), np.int64)
    for y in range(h // 2):
        for x in range(w // 2):
            s = 0
            for j in range(-2, 3):
                for i in range(-2, 3):
                    yy = min(max(2 * y + j, 0), h - 1)
                    xx = min(max(2 * x + i, 0), w - 1)
                    s += wts[i + 2] * wts[j + 2] * int(img[yy, xx])
            out[y, x] = (s + 128) >> 8
    return out


def test_pyramid_two_pass_equals_direct_sum():
    rng = np.random.default_rng(1)
    for h, w in ((17, 23), (20, 31)):
        img = rng.integers(0, 256, (h, w), dtype=np.uint8)
        assert (oracle.pyramid(img, 2)[1] == _direct_eq1(img)).all()


# --------------------------------------------------------------------------
# FAST-9 score (Sec. III-D)
# --------------------------------------------------------------------------

CIRCLE = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
          (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]


def _segment_test(img, x, y, tau):
    c = int(img[y, x])
    ring = [int(img[y + dy, x + dx]) for dx, dy in CIRCLE]
    for s in range(16):
        arc = [ring[(s + k) % 16] for k in range(9)]
        if all(v > c + tau for v in arc) or all(v < c - tau for v in arc):
            return True
    return False


def _brute_score(img, x, y):
    best = -1
    for tau in range(256):
        if _segment_test(img, x, y, tau):
            best = tau
    return best


def test_fast_score_matches_literal_segment_test():
    rng = np.random.default_rng(7)
    n = 0
    for trial in range(6):
        img = rng.integers(0, 256, (10, 10), dtype=np.uint8)
        if trial % 2:  # blocky images make long arcs and real corners
            img = np.kron(rng.integers(0, 256, (3, 3)), np.ones((4, 4)))[:10, :10].astype(np.uint8)
        s = oracle.fast_scores(img)
        for y in range(3, 7):
            for x in range(3, 7):
                assert s[y, x] == _brute_score(img, x, y), (trial, x, y)
                n += 1
    assert n == 96


def test_fast_early_out_pairs_cover_every_arc():
    # every 9-arc of the 16-circle contains one of {0, 8} and one of {4, 12}
    for s in range(16):
        arc = {(s + k) % 16 for k in range(9)}
        assert arc & {0, 8} and arc & {4, 12}


# --------------------------------------------------------------------------
# Detector (Sec. III-D)
# --------------------------------------------------------------------------


def _square(corner_bump=False):
    img = np.full((40, 40), 50, np.uint8)
    img[14:26, 14:26] = 200
    if corner_bump:
        for y, x in ((14, 14), (14, 25), (25, 14), (25, 25)):
            img[y, x] = 210
    return img


def test_uniform_square_is_a_plateau():
    # the four corner regions of a hard-edged square share equal scores, so a
    # strict 3x3 maximum finds nothing
    d = oracle.detect(_square(), 40, k=8, thresholds=(5,))
    assert (d[..., 2] < 0).all()


def test_square_with_bumped_corners():
    d = oracle.detect(_square(True), 40, k=8, thresholds=(5,))[0]
    found = sorted((int(x), int(y), int(s)) for x, y, s in d if s >= 0)
    # the bumped pixel (210) sees a 9-arc of background (50): score 210-50-1
    assert found == [(14, 14, 159), (14, 25, 159), (25, 14, 159), (25, 25, 159)]


def test_isolated_dot_score_is_contrast_minus_one():
    for contrast in (6, 40, 70, 205):
        img = np.full((20, 20), 50, np.uint8)
        img[10, 10] = 50 + contrast
        d = oracle.detect(img, 20, k=4, thresholds=(5,))[0]
        found = [(int(x), int(y), int(s)) for x, y, s in d if s >= 0]
        assert found == [(10, 10, contrast - 1)]


def test_threshold_walk_equals_single_pass():
    rng = np.random.default_rng(3)
    for trial in range(4):
        img = ndimage.zoom(rng.integers(0, 256, (12, 16)).astype(float), 4, order=0)
        img = np.clip(img + rng.normal(0, 8, img.shape), 0, 255).astype(np.uint8)
        for k in (1, 2, 3):
            a = oracle.detect(img, 16, k=k)
            b = oracle.detect(img, 16, k=k, single_pass=True)
            assert (a == b).all()


def _brute_cells(img, cell, k, tmin, margin):
    """Per-cell winners from the literal definitions, written independently."""
    h, w = img.shape
    S = np.full((h, w), -(1 << 30), np.int64)
    for y in range(3, h - 3):
        for x in range(3, w - 3):
            S[y, x] = _brute_score(img, x, y)
    ncx, ncy = -(-w // cell), -(-h // cell)
    out = []
    for cy in range(ncy):
        for cx in range(ncx):
            cands = []
            for y in range(cy * cell, min(h, cy * cell + cell)):
                for x in range(cx * cell, min(w, cx * cell + cell)):
                    if not (margin <= x <= w - 1 - margin and margin <= y <= h - 1 - margin):
                        continue
                    s = S[y, x]
                    if s < tmin:
                        continue
                    nb = S[y - 1:y + 2, x - 1:x + 2].copy()
                    nb[1, 1] = -(1 << 40)
                    if (s > nb).all():
                        cands.append((-s, y, x))
            cands.sort()
            out.append([(x, y, -ns) for ns, y, x in cands[:k]])
    return out


def test_cells_against_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(2):
        img = ndimage.zoom(rng.integers(0, 256, (6, 6)).astype(float), 6, order=0)[:32, :32]
        img = np.clip(img + rng.integers(-3, 4, img.shape), 0, 255).astype(np.uint8)
        for cell, k in ((8, 1), (16, 2), (11, 3)):
            got = oracle.detect(img, cell, k=k, margin=4)
            want = _brute_cells(img, cell, k, 5, 4)
            for c, wl in enumerate(want):
                g = [tuple(int(v) for v in r) for r in got[c] if r[2] >= 0]
                assert g == wl, (trial, cell, k, c)


# --------------------------------------------------------------------------
# Patch tracker (Sec. III-E, eqs. 4-5)
# --------------------------------------------------------------------------


def _smooth_texture(h, w, seed, sigma=2.0):
    rng = np.random.default_rng(seed)
    f = ndimage.gaussian_filter(rng.normal(0, 1, (h, w)), sigma)
    f = (f - f.min()) / (f.max() - f.min())
    return 30 + 190 * f


def test_pattern_is_the_52_point_disk():
    u, v = oracle.pattern()
    assert len(u) == 52
    pts = set(zip(u.tolist(), v.tolist()))
    want = {(a + 0.5, b + 0.5) for a in range(-4, 4) for b in range(-4, 4)
            if (a + 0.5) ** 2 + (b + 0.5) ** 2 <= 16}
    assert pts == want and len(want) == 52
    order = list(zip(v.tolist(), u.tolist()))
    assert order == sorted(order)


def test_se2_exp_identities():
    # exp(t, 0) is a pure translation; exp(d) exp(-d) = identity
    assert oracle.se2_exp(1.5, -2.0, 0.0) == (1.5, -2.0)
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b, phi = rng.normal(0, 2), rng.normal(0, 2), rng.uniform(-1, 1)
        tx, ty = oracle.se2_exp(a, b, phi)
        ux, uy = oracle.se2_exp(-a, -b, -phi)
        # compose (R(phi), t) with (R(-phi), u): t + R(phi) u
        c, s = math.cos(phi), math.sin(phi)
        assert abs(tx + c * ux - s * uy) < 1e-12 and abs(ty + s * ux + c * uy) < 1e-12
        # against the matrix exponential of the se(2) generator
        from scipy.linalg import expm
        M = expm(np.array([[0, -phi, a], [phi, 0, b], [0, 0, 0]]))
        assert abs(M[0, 2] - tx) < 1e-10 and abs(M[1, 2] - ty) < 1e-10
    # small-angle branch agrees with the closed form
    tx, ty = oracle.se2_exp(1.0, 2.0, 5e-5)
    M = __import__("scipy.linalg", fromlist=["expm"]).expm(np.array([[0, -5e-5, 1.0], [5e-5, 0, 2.0], [0, 0, 0]]))
    assert abs(M[0, 2] - tx) < 1e-12 and abs(M[1, 2] - ty) < 1e-12


def test_inverse3_against_solve():
    rng = np.random.default_rng(2)
    for _ in range(20):
        A = rng.normal(size=(3, 3))
        A = A @ A.T + 0.1 * np.eye(3)
        det, inv = oracle.inverse3(A.ravel())
        assert abs(det - np.linalg.det(A)) < 1e-9 * max(1, abs(det))
        assert np.allclose(inv, np.linalg.solve(A, np.eye(3)), rtol=1e-9, atol=1e-12)


def test_template_hessian_against_direct_jacobian():
    img = np.round(_smooth_texture(40, 40, 3)).astype(np.uint8)
    H, Hinv, fits, valid = oracle.template(img, 20.25, 19.5)
    assert fits and valid
    # Jacobian rows from central differences of bilinear samples, mean-normalised
    u, v = oracle.pattern()
    f = img.astype(np.float64)

    def bil(x, y):
        return ndimage.map_coordinates(f, [[y], [x]], order=1)[0]
    I = np.array([bil(20.25 + a, 19.5 + b) for a, b in zip(u, v)])
    m = I.mean()
    gx = np.array([(bil(20.25 + a + 1, 19.5 + b) - bil(20.25 + a - 1, 19.5 + b)) / 2 for a, b in zip(u, v)]) / m
    gy = np.array([(bil(20.25 + a, 19.5 + b + 1) - bil(20.25 + a, 19.5 + b - 1)) / 2 for a, b in zip(u, v)]) / m
    J = np.stack([gx, gy, gy * u - gx * v], 1)
    assert np.allclose(H, J.T @ J, rtol=1e-9)
    assert np.allclose(Hinv @ H, np.eye(3), atol=1e-9)


def test_flat_and_ramp_patches_are_degenerate():
    flat = np.full((48, 48), 100, np.uint8)
    _, st = oracle.track(flat, flat, [[24, 24]], [[24, 24]], 1, 5)
    assert st[0] == oracle.LOST_DEGENERATE
    yy, xx = np.mgrid[0:48, 0:48]
    ramp = (2 * xx + 3 * yy + 10).astype(np.uint8)
    H, _, fits, valid = oracle.template(ramp, 24, 24)
    assert fits and not valid  # rank-2 Hessian (aperture problem)
    _, st = oracle.track(ramp, ramp, [[24, 24]], [[24, 24]], 1, 5)
    assert st[0] == oracle.LOST_DEGENERATE


def test_identical_frames_give_zero_motion_exactly():
    img = synthgen.sequence(synthgen.WORKLOADS["mono320"]).frames[0, 0]
    pts = np.array([[100.0, 80.0], [160.5, 120.25], [33.0, 200.0], [250.0, 40.0]])
    for dbl in (False, True):
        out, st = oracle.track(img, img, pts, pts, 3, 5, double=dbl)
        assert (st == oracle.TRACKED).all()
        assert (out[:, :2] == pts).all() and (out[:, 3] == 0).all() and (out[:, 2] == 0).all()


def test_integer_translation_recovered():
    tex = np.round(_smooth_texture(128, 128, 4)).astype(np.uint8)
    dx, dy = 4, -8  # multiples of 2^(L-1): the shift is exact at every level
    dst = np.roll(tex, (dy, dx), axis=(0, 1))
    pts = np.array([[60.0, 60.0], [64.5, 70.25], [50.0, 55.0]])
    init = pts + [dx + 0.7, dy - 0.6]
    out = oracle.klt_pass(tex, dst, pts, init, 3, 10)
    assert (out[:, 5] == 0).all()
    assert np.abs(out[:, 0] - (pts[:, 0] + dx)).max() < 1e-4
    assert np.abs(out[:, 1] - (pts[:, 1] + dy)).max() < 1e-4
    assert np.abs(out[:, 2]).max() < 1e-5
    assert out[:, 3].max() < 1e-6  # residual vanishes at the solution


def _warp(tex, tx, ty, th, c):
    h, w = tex.shape
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    cs, sn = math.cos(th), math.sin(th)
    dx, dy = xx - c[0] - tx, yy - c[1] - ty
    sx, sy = c[0] + cs * dx + sn * dy, c[1] - sn * dx + cs * dy
    return ndimage.map_coordinates(tex, [sy, sx], order=3, mode="nearest")


def test_subpixel_se2_recovered_on_smooth_texture():
    tex = _smooth_texture(160, 160, 9, sigma=2.5)
    c = (80.0, 80.0)
    rng = np.random.default_rng(9)
    errs = []
    for trial in range(4):
        tx, ty, th = rng.uniform(-2, 2), rng.uniform(-2, 2), math.radians(rng.uniform(-1.5, 1.5))
        src = np.round(tex).astype(np.uint8)
        dst = np.clip(np.round(_warp(tex, tx, ty, th, c)), 0, 255).astype(np.uint8)
        pts = rng.uniform(40, 120, (25, 2))
        gx = c[0] + math.cos(th) * (pts[:, 0] - c[0]) - math.sin(th) * (pts[:, 1] - c[1]) + tx
        gy = c[1] + math.sin(th) * (pts[:, 0] - c[0]) + math.cos(th) * (pts[:, 1] - c[1]) + ty
        out, st = oracle.track(src, dst, pts, pts, 3, 5, fb_threshold=0.3)
        ok = st == oracle.TRACKED
        assert ok.mean() > 0.9
        errs.append(np.hypot(out[ok, 0] - gx[ok], out[ok, 1] - gy[ok]))
        # the patch rotation estimate follows the true rotation
        assert abs(np.median(out[ok, 2]) - th) < math.radians(0.3)
    # The floor here is u8 quantisation: on a smooth texture the rounding error
    # is correlated across the 52 samples and does not average out (a smoother
    # texture makes it worse, not better). Gross slips (a sign, a transposed
    # rotation, a wrong level scale) give errors of a pixel or more; the tight
    # pins are the exact integer shift and the brute-force SSD minimum.
    e = np.concatenate(errs)
    assert np.median(e) <= 0.05 and np.percentile(e, 95) <= 0.1


def test_klt_lands_on_brute_force_ssd_minimum():
    """Gauss-Newton converges to the grid minimum of the eq. (4) residual."""
    tex = _smooth_texture(48, 48, 21, sigma=1.8)
    src = np.round(tex).astype(np.uint8)
    dst = np.clip(np.round(_warp(tex, 0.37, -0.81, math.radians(0.6), (24.0, 24.0))), 0, 255).astype(np.uint8)
    u, v = oracle.pattern()
    u, v = u.astype(np.float64), v.astype(np.float64)
    p = np.array([24.0, 24.0])
    fs, fd = src.astype(np.float64), dst.astype(np.float64)

    def bil(f, x, y):
        return ndimage.map_coordinates(f, [y, x], order=1)
    T = bil(fs, p[0] + u, p[1] + v)
    T = T / T.mean()

    def ssd(tx, ty, th):
        c, s = np.cos(th), np.sin(th)
        wx = c[..., None] * u - s[..., None] * v + tx[..., None]
        wy = s[..., None] * u + c[..., None] * v + ty[..., None]
        I = bil(fd, wx.ravel(), wy.ravel()).reshape(wx.shape)
        e = I / I.mean(-1, keepdims=True) - T
        return (e * e).sum(-1)

    def grid(cx, cy, cth, half, step, thalf, tstep):
        ax = np.arange(-half, half + 1e-9, step)
        at = np.arange(-thalf, thalf + 1e-12, tstep)
        X, Y, TH = np.meshgrid(cx + ax, cy + ax, cth + at, indexing="ij")
        f = ssd(X.ravel(), Y.ravel(), TH.ravel())
        i = int(np.argmin(f))
        return X.ravel()[i], Y.ravel()[i], TH.ravel()[i]
    bx, by, bt = grid(p[0], p[1], 0.0, 2.0, 0.1, math.radians(2), math.radians(0.25))
    bx, by, bt = grid(bx, by, bt, 0.15, 0.01, math.radians(0.3), math.radians(0.05))
    out = oracle.klt_pass(src, dst, [p], [p], 1, 20)
    assert out[0, 5] == 0
    # the inverse-compositional fixed point (template gradients) and the SSD
    # minimum (target gradients) coincide only at zero residual; with u8
    # rounding they differ by O(residual), here about 0.01 px, plus the 0.01-px
    # grid step
    assert abs(out[0, 0] - bx) <= 0.02 and abs(out[0, 1] - by) <= 0.02
    assert abs(out[0, 2] - bt) <= math.radians(0.1)
    assert out[0, 4] < 1e-4  # the last step is small once converged


# Level schedule and image domain (Sec. III-E; the paper is silent on borders).
# Reading: a coarse level whose template does not fit is skipped, with t still
# doubled through it; the template fits when every sample and its +-1 px
# gradient neighbours lie in the closed domain [0, W-1] x [0, H-1]; a warped
# sample outside that domain, or a template that does not fit at level 0, is
# LOST_OOB.


def test_coarse_level_that_does_not_fit_is_skipped():
    tex = np.round(_smooth_texture(128, 128, 4)).astype(np.uint8)
    dx, dy = 4, -8
    dst = np.roll(tex, (dy, dx), axis=(0, 1))
    # x = 8.98: level 1 holds the keypoint at 4.49, where the pattern's
    # leftmost gradient tap (4.49 - 3.5 - 1) falls outside the image; level 0
    # (8.98 - 4.5 >= 0) fits. Skipping the coarse levels leaves t = init at
    # level 0, so the 2- and 3-level passes equal the 1-level pass bit for bit.
    p = np.array([[8.98, 64.0]])
    init = p + [dx + 0.3, dy - 0.2]
    one = oracle.klt_pass(tex, dst, p, init, 1, 10)
    assert one[0, 5] == oracle.TRACKED
    assert abs(one[0, 0] - (p[0, 0] + dx)) < 1e-2 and abs(one[0, 1] - (p[0, 1] + dy)) < 1e-2
    for L in (2, 3):
        out = oracle.klt_pass(tex, dst, p, init, L, 10)
        assert out[0, 5] == oracle.TRACKED, L
        assert (out[0, :5] == one[0, :5]).all(), (L, out[0], one[0])
    # x = 9.0: level 1 (4.5) fits and is used, so the 2-level pass differs
    q = np.array([[9.0, 64.0]])
    two = oracle.klt_pass(tex, dst, q, q + [dx + 0.3, dy - 0.2], 2, 10)
    lone = oracle.klt_pass(tex, dst, q, q + [dx + 0.3, dy - 0.2], 1, 10)
    assert two[0, 5] == oracle.TRACKED and (two[0, :3] != lone[0, :3]).any()
    # the full forward-backward tracker keeps the near-border keypoint
    out, st = oracle.track(tex, dst, p, init, 3, 5)
    assert st[0] == oracle.TRACKED and abs(out[0, 0] - (p[0, 0] + dx)) < 5e-2


@pytest.mark.parametrize("axis", [0, 1])
def test_template_fit_boundary(axis):
    """The template fits iff the outermost gradient tap (3.5 + 1 px from the
    keypoint) lies in [0, W-1]: at level 0 alone a misfit is LOST_OOB."""
    tex = np.round(_smooth_texture(96, 128, 6)).astype(np.uint8)  # H 96, W 128
    size = tex.shape[1 - axis]
    for c, fits in ((4.5, True), (4.49, False), (size - 1 - 4.5, True), (size - 1 - 4.49, False)):
        p = np.array([[c, 48.0]] if axis == 0 else [[64.0, c]])
        out = oracle.klt_pass(tex, tex, p, p, 1, 1)
        assert out[0, 5] == (oracle.TRACKED if fits else oracle.LOST_OOB), (c, out[0])
        _, st = oracle.track(tex, tex, p, p, 1, 1)
        assert st[0] == (oracle.TRACKED if fits else oracle.LOST_OOB), c


def test_warp_leaving_the_image_is_lost_oob():
    tex = np.round(_smooth_texture(128, 128, 8)).astype(np.uint8)
    p = np.array([[64.0, 64.0]])
    # first iteration's warp at the start: the pattern reaches 3.5 px from it;
    # the closed domain admits a sample exactly on the first or last column
    for sx, ok in ((3.5, True), (3.49, False), (127 - 3.5, True), (127 - 3.49, False)):
        out = oracle.klt_pass(tex, tex, p, [[sx, 64.0]], 1, 1)
        assert out[0, 5] == (oracle.TRACKED if ok else oracle.LOST_OOB), (sx, out[0])
        out = oracle.klt_pass(tex, tex, p, [[64.0, sx]], 1, 1)
        assert out[0, 5] == (oracle.TRACKED if ok else oracle.LOST_OOB), (sx, out[0])
    # a keypoint whose true match lies past the border: src is dst shifted so
    # that the match of x = 12 sits at x = 1, and the converging warp leaves
    # the image; clamped addressing would return a position instead
    dst = np.ascontiguousarray(np.concatenate([tex[:, 11:], tex[:, :11]], 1))
    q = np.array([[12.0, 64.0]])
    out = oracle.klt_pass(tex, dst, q, q - [8.0, 0.0], 1, 20)
    assert out[0, 5] == oracle.LOST_OOB, out[0]
    _, st = oracle.track(tex, dst, q, q - [8.0, 0.0], 1, 20)
    assert st[0] == oracle.LOST_OOB


def test_backward_pass_starts_from_the_inverse_of_the_forward_motion():
    """Fig. 4: the backward pass rebuilds the template on the target at the
    forward result p' and starts from the inverse motion, position p and
    rotation -theta_fwd. When the forward pass starts at the true motion (a
    20 degree rotation about the image centre plus a shift), that start is
    already the backward solution, so a single Gauss-Newton iteration per pass
    returns to p: the forward-backward distance stays at the interpolation
    level. A start at +theta_fwd (40 degrees off) or at p' (a full re-track)
    cannot get back in one iteration."""
    tex = _smooth_texture(160, 160, 11, sigma=2.0)
    th, d, c = math.radians(20.0), (2.0, -1.5), (80.0, 80.0)
    src = np.round(tex).astype(np.uint8)
    dst = np.clip(np.round(_warp(tex, d[0], d[1], th, c)), 0, 255).astype(np.uint8)
    pts = np.random.default_rng(3).uniform(50, 110, (20, 2))
    gx = c[0] + math.cos(th) * (pts[:, 0] - c[0]) - math.sin(th) * (pts[:, 1] - c[1]) + d[0]
    gy = c[1] + math.sin(th) * (pts[:, 0] - c[0]) + math.cos(th) * (pts[:, 1] - c[1]) + d[1]
    for dbl in (False, True):
        out, st = oracle.track(src, dst, pts, np.stack([gx, gy], 1), 1, 1, fb_threshold=0.3, double=dbl, theta0=th)
        assert (st == oracle.TRACKED).all(), st
        assert np.median(out[:, 3]) < 0.05 and out[:, 3].max() < 0.1, np.sort(out[:, 3])


def test_float_and_double_trackers_agree():
    seq = synthgen.sequence(synthgen.WORKLOADS["mono320"])
    d = oracle.detect(seq.frames[0, 0], 16)[:, 0]
    pts = d[d[:, 2] >= 0, :2].astype(np.float64)
    a, sa = oracle.track(seq.frames[0, 0], seq.frames[1, 0], pts, pts, 3, 5, double=False)
    b, sb = oracle.track(seq.frames[0, 0], seq.frames[1, 0], pts, pts, 3, 5, double=True)
    both = (sa == oracle.TRACKED) & (sb == oracle.TRACKED)
    assert both.mean() > 0.9
    assert np.abs(a[both, :2] - b[both, :2]).max() < 1e-3


# --------------------------------------------------------------------------
# Pipeline (Sec. III-B) on the synthetic workloads
# --------------------------------------------------------------------------


def test_mono_pipeline_accuracy_against_ground_truth():
    w = synthgen.WORKLOADS["mono320"]
    seq = synthgen.sequence(w)
    fe = oracle.Frontend([w.width], [w.height], False, oracle.params_for(w))
    fe.push([seq.frames[0, 0]])
    r0 = fe.records()
    assert (r0["status"] == oracle.DETECTED).all() and len(r0) > 50
    assert (np.diff(r0["id"]) > 0).all()
    fe.push([seq.frames[1, 0]])
    r1 = fe.records()
    tr = r1[r1["status"] == oracle.TRACKED]
    assert len(tr) >= 0.95 * len(r0)
    src = {int(i): (x, y) for i, x, y in zip(r0["id"], r0["x"], r0["y"])}
    px = np.array([src[int(i)][0] for i in tr["id"]])
    py = np.array([src[int(i)][1] for i in tr["id"]])
    gx, gy = seq.gt_temporal(0, 0, px, py)
    err = np.hypot(tr["x"] - gx, tr["y"] - gy)
    assert np.median(err) <= 0.1
    assert len(r1) <= w.max_keypoints + len(r0)


def test_selection_rules_mask_cap_and_ids():
    """New keypoints = unmasked cell winners, best first up to the cap, ids in cell order."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, n_frames=1)
    img = seq.frames[0, 0]
    cell = w.cell_size
    win = oracle.detect(img, cell)[:, 0]
    ncx = -(-w.width // cell)
    rng = np.random.default_rng(0)
    for live_n, cap in ((0, 300), (40, 100), (150, 160)):
        params = oracle.params_for(w, max_keypoints=cap)
        fe = oracle.Frontend([w.width], [w.height], False, params)
        # live keypoints placed at random positions, injected as the host would
        xy = rng.uniform(10, [w.width - 10, w.height - 10], (live_n, 2)).astype(np.float32)
        fe.set_keypoints(0, np.arange(live_n), xy, xy, np.zeros(live_n))
        # the first frame has no previous pyramid: the injected keypoints are
        # kept as they are and mask their cells
        fe.push([img])
        r = fe.records()
        new = r[r["status"] == oracle.DETECTED]
        occ = np.zeros(len(win), int)
        for x, y in xy:
            occ[int(np.floor(y / cell)) * ncx + int(np.floor(x / cell))] += 1
        cands = [(-int(win[c, 2]), c) for c in range(len(win)) if win[c, 2] >= 0 and occ[c] == 0]
        cands.sort()
        room = max(0, cap - live_n)
        chosen = sorted(c for _, c in cands[:room])
        assert [(int(x), int(y)) for x, y in zip(new["x"], new["y"])] == \
            [(int(win[c, 0]), int(win[c, 1])) for c in chosen]
        assert list(new["id"]) == list(range(live_n, live_n + len(chosen)))
        assert list(new["score"]) == [int(win[c, 2]) for c in chosen]
