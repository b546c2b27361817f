"""Pins of the oracle's Kannala-Brandt equidistant fisheye model (KB4: a ray at
angle theta to the optical axis lands at radius theta (1 + k1 theta^2 + ... +
k4 theta^8) on the normalised image plane) as the camera model of the
camera-model start (Sec. III-E), against closed forms: the equidistant special
case, the pinhole model through the Taylor series of tan, rotations about the
optical axis, and the inverse-distance convention of a fisheye ray."""
import numpy as np
import pytest

import oracle
import synthgen

F, CX, CY = 400.0, 375.5, 239.5
# the Taylor coefficients of tan(theta) = theta + theta^3/3 + 2 theta^5/15 + 17 theta^7/315 + 62 theta^9/2835 + ...
TAN4 = (1 / 3, 2 / 15, 17 / 315, 62 / 2835)
KB_TAN = (F, F, CX, CY, *TAN4)
KB_EQ = (F, F, CX, CY, 0.0, 0.0, 0.0, 0.0)


def _ray(theta, phi):
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)


def test_equidistant_radius_is_focal_times_angle():
    """k = 0: the pixel radius is f theta, also for rays beyond 90 degrees."""
    th = np.array([0.0, 0.1, 0.7, 1.4, 2.0, 2.9])
    ph = np.array([0.3, -1.0, 2.0, 0.5, -2.5, 1.2])
    out, ok = oracle.camera_project(KB_EQ, _ray(th, ph) * 3.0)
    assert ok.all()
    np.testing.assert_allclose(out[:, 0], CX + F * th * np.cos(ph), atol=1e-9)
    np.testing.assert_allclose(out[:, 1], CY + F * th * np.sin(ph), atol=1e-9)
    # a point on the axis behind the camera has no pixel
    _, ok = oracle.camera_project(KB_EQ, [[0.0, 0.0, -1.0]])
    assert not ok[0]


def test_tan_series_coefficients_reproduce_the_pinhole_model():
    """With the first four Taylor coefficients of tan, KB4 differs from the
    pinhole projection by the series remainder, below 2 * 1382/155925 theta^11
    in normalised units for theta <= 0.6."""
    r = np.random.default_rng(3)
    th, ph = r.uniform(0.0, 0.6, 400), r.uniform(-np.pi, np.pi, 400)
    X = _ray(th, ph) * r.uniform(0.5, 5.0, (400, 1))
    kb, ok1 = oracle.camera_project(KB_TAN, X)
    pin, ok2 = oracle.camera_project((F, F, CX, CY), X)
    assert ok1.all() and ok2.all()
    err = np.hypot(*(kb - pin).T)
    assert (err <= F * 2 * 1382 / 155925 * th ** 11 + 1e-9).all(), err.max()
    # a wrong coefficient (k1 and k2 swapped) is far off at the same angles
    bad, _ = oracle.camera_project((F, F, CX, CY, TAN4[1], TAN4[0], TAN4[2], TAN4[3]), X)
    assert np.hypot(*(bad - pin).T).max() > 1.0


@pytest.mark.parametrize("k", [TAN4, (0.0, 0.0, 0.0, 0.0), (-0.02, 0.004, -0.001, 0.0002), (0.05, -0.01, 0.0, 0.0)])
def test_unprojection_inverts_the_projection(k):
    """Newton's inversion of the radius polynomial: unprojecting and projecting
    again returns the pixel, the point lies at distance 1 (inverse depth 1) on
    the ray, and the ray's angle is the one whose radius is the pixel's."""
    K = (F, F * 1.01, CX, CY, *k)
    r = np.random.default_rng(7)
    pts = np.stack([r.uniform(0, 751, 300), r.uniform(0, 479, 300)], 1)
    pts[0] = (CX, CY)  # the optical axis
    back, rays, ok = oracle.camera_roundtrip(K, pts)
    assert ok.all()
    np.testing.assert_allclose(back, pts, atol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(rays, axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(rays[0], [0, 0, 1], atol=1e-15)
    # the ray's pixel by the equidistant map of the KB4 radius, stated with numpy
    th = np.arccos(np.clip(rays[:, 2], -1, 1))
    rad = th * (1 + k[0] * th ** 2 + k[1] * th ** 4 + k[2] * th ** 6 + k[3] * th ** 8)
    rn = np.hypot((pts[:, 0] - CX) / K[0], (pts[:, 1] - CY) / K[1])
    np.testing.assert_allclose(rad, rn, atol=1e-9)


def test_back_projection_near_the_fold_of_the_radius_polynomial():
    """k = (-0.3, 0, 0, 0): r(theta) = theta - 0.3 theta^3 rises to its fold at
    theta = 1/sqrt(0.9) (r = 0.70273) with slope r' = 1 - 0.9 theta^2. A pixel
    whose root has slope >= 0.05 has a ray (the root of the cubic, from
    numpy's polynomial roots); at slope 0.04, at the fold and beyond it (no
    root at all) the back-projection is refused."""
    K = (F, F, CX, CY, -0.3, 0.0, 0.0, 0.0)
    for slope, want in ((0.5, True), (0.06, True), (0.04, False), (0.0, False)):
        th = np.sqrt((1 - slope) / 0.9)
        td = th - 0.3 * th ** 3
        px = [[CX + F * td * np.cos(0.7), CY + F * td * np.sin(0.7)]]
        out, rays, ok = oracle.camera_roundtrip(K, px)
        assert ok[0] == want, (slope, ok[0])
        if want:
            roots = np.roots([-0.3, 0.0, 1.0, -td])
            root = min(r.real for r in roots if abs(r.imag) < 1e-12 and r.real >= 0)
            assert abs(np.arccos(rays[0, 2] / np.linalg.norm(rays[0])) - root) < 1e-9
            np.testing.assert_allclose(out[0], px[0], atol=1e-7)
    # beyond the fold (r > 0.70273 has no root)
    _, _, ok = oracle.camera_roundtrip(K, [[CX + F * 0.71, CY]])
    assert not ok[0]


def test_roll_about_the_optical_axis_rotates_the_pixels():
    """KB4 is symmetric about the optical axis: a roll by phi (R = Rz(phi),
    t = 0, fx = fy) rotates every pixel by phi about the principal point and
    starts the warp at angle phi, at any inverse depth."""
    phi = 0.21
    R = np.array([[np.cos(phi), -np.sin(phi), 0], [np.sin(phi), np.cos(phi), 0], [0, 0, 1]])
    r = np.random.default_rng(1)
    pts = np.stack([r.uniform(40, 710, 100), r.uniform(30, 450, 100)], 1)
    out, ok = oracle.motion_start((F, F, CX, CY, -0.02, 0.004, -0.001, 0.0002), R, np.zeros(3), pts,
                                  r.uniform(0.1, 3.0, 100))
    assert ok.all()
    d = pts - [CX, CY]
    want = np.stack([np.cos(phi) * d[:, 0] - np.sin(phi) * d[:, 1], np.sin(phi) * d[:, 0] + np.cos(phi) * d[:, 1]], 1)
    np.testing.assert_allclose(out[:, :2], want + [CX, CY], atol=1e-8)
    np.testing.assert_allclose(out[:, 2], phi, atol=1e-6)


def test_fisheye_inverse_depth_is_inverse_distance_along_the_ray():
    """A pixel at angle theta0 from the axis (k = 0, on the x axis) at inverse
    depth rho is the point (sin theta0, 0, cos theta0) / rho; moving the camera
    forward by half that point's depth puts it at angle
    atan2(sin theta0, cos theta0 / 2)."""
    th0, rho = 0.8, 0.4
    px = np.array([[CX + F * th0, CY]])
    t = [0.0, 0.0, -0.5 * np.cos(th0) / rho]
    out, ok = oracle.motion_start(KB_EQ, np.eye(3), t, px, rho)
    assert ok.all()
    np.testing.assert_allclose(out[0, :2], [CX + F * np.arctan2(np.sin(th0), 0.5 * np.cos(th0)), CY], atol=1e-9)
    # the pinhole model's inverse depth is along the optical axis: the same
    # step moves its point at depth 1 / rho (not distance) to half that depth
    pin, ok = oracle.motion_start((F, F, CX, CY), np.eye(3), t, [[CX + F * 0.5, CY]], rho)
    z = 1 / rho - 0.5 * np.cos(th0) / rho
    np.testing.assert_allclose(pin[0, 0], CX + F * (0.5 / rho) / z, atol=1e-9)


def test_projection_between_a_pinhole_and_a_fisheye_camera():
    """Stereo extrinsics mix models: back-projecting through the pinhole
    camera and projecting through a KB4 camera with the tan coefficients lands
    within the series remainder of the pinhole-to-pinhole projection."""
    R = np.eye(3)
    t = [-0.11, 0.0, 0.0]
    r = np.random.default_rng(2)
    pts = np.stack([r.uniform(200, 550, 50), r.uniform(100, 380, 50)], 1)
    a, ok1 = oracle.motion_start((F, F, CX, CY), R, t, pts, 0.5, Kq=KB_TAN)
    b, ok2 = oracle.motion_start((F, F, CX, CY), R, t, pts, 0.5)
    assert ok1.all() and ok2.all()
    assert np.abs(a[:, :2] - b[:, :2]).max() < 2e-3
    assert np.abs(a[:, 2] - b[:, 2]).max() < 1e-4


def _pipeline(K, frames=4, at=2):
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=6, n_frames=frames)
    fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
    out = []
    try:
        for t in range(frames):
            if t == at and K is not None:
                Kp, R, tr = seq.camera_motion(t - 1, 460.0, 0.4)
                Kc = Kp if len(K) == 0 else (*Kp, *K)
                fe.set_motion(0, Kc, R, tr, 0.4)
            fe.push(list(seq.frames[t]))
            out.append(fe.records())
    finally:
        fe.close()
    return out


def test_pipeline_fisheye_model_with_tan_coefficients_tracks_like_the_pinhole():
    """Wired through the frame pipeline: the KB4 model with the tan series
    starts the tracks within the series remainder of the pinhole start (up to
    about 0.2 px in the image corners at f = 460), and the tracker takes them
    to the same statuses and, but for a few weak corners, the same positions
    within 1e-3 px."""
    kb, pin, plain = _pipeline(TAN4), _pipeline(()), _pipeline(None)
    a, b = kb[2], pin[2]
    assert (a["id"] == b["id"]).all() and (a["status"] == b["status"]).all()
    ok = a["status"] == oracle.TRACKED
    assert ok.sum() > 50
    d = np.maximum(np.abs(a["x"][ok] - b["x"][ok]), np.abs(a["y"][ok] - b["y"][ok]))
    assert (d < 1e-3).mean() >= 0.95 and d.max() < 0.05, (np.sort(d)[-5:], (d < 1e-3).mean())
    # and the model was used: the start differs from constant velocity's
    assert a.tobytes() != plain[2].tobytes()


def test_invalid_models_are_refused():
    with pytest.raises(AssertionError):
        oracle.camera_project((F, F, CX), [[0, 0, 1.0]])
    with pytest.raises(AssertionError):
        oracle.camera_project((F, F, CX, CY, np.nan, 0, 0, 0), [[0, 0, 1.0]])
