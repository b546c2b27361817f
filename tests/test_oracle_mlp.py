"""Pins of the oracle's learned-initialisation part (MLP, loss, Adam, features).

The MLP is a project addition, not part of the paper; these checks tie the
oracle to mathematics that fixes it: bfloat16 rounding against torch's own
conversion, the backward pass against FP64 central differences, the loss and
Adam against closed forms, and the features against hand-built cases.
"""
import math

import numpy as np
import pytest

import oracle


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.normal(0, 3, 2000), rng.normal(0, 1e-30, 200), rng.normal(0, 1e30, 200),
                           [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.0078125, 3.0e38, -1e-45, 65504.0]])
    vals = vals.astype(np.float32)
    want = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle.bf16(v) for v in vals], np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def _batch(n=48, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 0.6, (n, 32)).astype(np.float32)
    T = rng.normal(0, 1.5, (n, 2)).astype(np.float32)
    return X, T


def test_loss_closed_form():
    # zero weights: y = b3 for every sample
    P = np.zeros(oracle.MLP_NPARAM, np.float32)
    P[-3:] = [0.125, -0.0625, 0.5]          # guess (2, -1) px, logit 0.5
    X = np.zeros((1, 32), np.float32)
    T = np.array([[2.5, -4.0]], np.float32)  # errors -0.5 (quadratic) and 3 (linear)
    L, G, dY = oracle.mlp_loss_grad(P, X, T, exact=True)
    c = 0.0                                  # |(-0.5, 3)| > 2 px
    bce = math.log1p(math.exp(0.5)) - c * 0.5
    assert abs(L - (0.5 * 0.25 + (3 - 0.5) + bce)) < 1e-12
    assert np.allclose(dY[0], [16 * -0.5, 16 * 1.0, 1 / (1 + math.exp(-0.5)) - c])


def test_gradient_against_fp64_central_differences():
    P = oracle.mlp_init(3)
    P[oracle.MLP_NPARAM - 3:] = 0.01
    X, T = _batch()
    _, G, _ = oracle.mlp_loss_grad(P, X, T, exact=True)
    rng = np.random.default_rng(4)
    # sample from every block: W1, b1, W2, b2, W3, b3
    blocks = [(0, 4096), (4096, 4224), (4224, 20608), (20608, 20736), (20736, 21120), (21120, 21123)]
    idx = np.concatenate([rng.choice(np.arange(a, b), min(b - a, 60), replace=False) for a, b in blocks])
    rel = []
    for i in idx:
        # small enough that no ReLU or Huber kink of the batch falls inside +-h
        h = 2e-6 * max(1.0, abs(float(P[i])))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] = np.float32(P[i] + h)
        Pm[i] = np.float32(P[i] - h)
        step = float(Pp[i]) - float(Pm[i])   # the perturbation actually representable in float
        Lp = oracle.mlp_loss_grad(Pp, X, T, exact=True)[0]
        Lm = oracle.mlp_loss_grad(Pm, X, T, exact=True)[0]
        fd = (Lp - Lm) / step
        if abs(G[i]) < 1e-7 and abs(fd) < 1e-7:
            continue
        rel.append(abs(fd - G[i]) / max(abs(G[i]), abs(fd), 1e-9))
    rel = np.array(rel)
    assert len(rel) > 200
    # a kink inside +-h would spoil a central difference; allow the odd one
    assert np.mean(rel < 1e-4) > 0.98, np.sort(rel)[-10:]
    assert np.median(rel) < 1e-6


def _one_path_net(paths, b3=(0.0, 0.0, 0.0)):
    """Parameters of a network whose output c is one chain input i -> h1 unit
    j -> h2 unit j -> y c: paths = [(i, j, c, w1, b1, w2, b2, w3)]."""
    P = np.zeros(oracle.MLP_NPARAM, np.float32)
    W1, B1 = 0, 128 * 32
    W2, B2 = B1 + 128, B1 + 128 + 128 * 128
    W3, B3 = B2 + 128, B2 + 128 + 3 * 128
    for i, j, c, w1, b1, w2, b2, w3 in paths:
        P[W1 + j * 32 + i], P[B1 + j] = w1, b1
        P[W2 + j * 128 + j], P[B2 + j] = w2, b2
        P[W3 + c * 128 + j] = w3
    P[B3:B3 + 3] = b3
    return P


def test_bf16_rounding_points_hand_derived():
    """The GPU's rounding points, one at a time, on hand-built one-path
    networks; every expected value below is worked out by hand from the
    bfloat16 grid (8 significant bits: next to 1 the spacing is 2^-7, and
    1 + 2^-8 is the tie between 1 and 1 + 2^-7, which goes to the even 1).

    Network A (weights and activations):
      w1 = 1 + 2^-9 rounds to 1; x = 1; b1 = 3 * 2^-10: 1 + 3 * 2^-10 lies
      below the tie 1 + 2^-8, so h1 = 1. Same for layer 2: h2 = 1. w3 = 1 +
      2^-9 rounds to 1; y0 = 1 + b3[0] with b3[0] = 2^-12 + 2^-21 kept in
      float (bfloat16 would drop the 2^-21), and y is not rounded.
      Slips: unrounded weights give h1 = bf16(1 + 2^-9 + 3 * 2^-10) = 1 + 2^-7;
      an unrounded h1 makes h2 = bf16(1 + 6 * 2^-10) = 1 + 2^-7; an unrounded
      h2 gives y0 = 1 + 3 * 2^-10 + ...; a rounded y gives 1.
    Network B (inputs and biases):
      path 0: x0 = 1 + 2^-9 rounds to 1, + b1 = 3 * 2^-10 -> h1 = 1 -> y0 = 1
      (an unrounded input gives 1 + 5 * 2^-10, above the tie: 1 + 2^-7);
      path 1: x1 = 1, b1 = 2^-8 + 2^-20 (float): 1 + 2^-8 + 2^-20 lies above
      the tie -> 1 + 2^-7 = y1 (a bias rounded to 2^-8 lands on the tie: 1);
      path 2: x2 = 0.75, h1 = 0.75, w2 = -1, b2 = 0.5: relu(-0.25) = 0, so
      y2 = b3[2] = 0.1 in float (rounding the pre-activation first would not
      change it; dropping the ReLU gives -0.25 + 0.1)."""
    A = _one_path_net([(0, 0, 0, 1 + 2 ** -9, 3 * 2 ** -10, 1.0, 3 * 2 ** -10, 1 + 2 ** -9)],
                      b3=(2 ** -12 + 2 ** -21, 0.1, -0.3))
    X = np.zeros((1, 32), np.float32)
    X[0, 0] = 1.0
    Y, H1, H2 = oracle.mlp_forward(A, X)
    assert H1[0, 0] == 1.0 and H2[0, 0] == 1.0
    assert Y[0, 0] == np.float32(1 + 2 ** -12 + 2 ** -21)
    assert Y[0, 1] == np.float32(0.1) and Y[0, 2] == np.float32(-0.3)
    B = _one_path_net([(0, 0, 0, 1.0, 3 * 2 ** -10, 1.0, 0.0, 1.0),
                       (1, 1, 1, 1.0, 2 ** -8 + 2 ** -20, 1.0, 0.0, 1.0),
                       (2, 2, 2, 1.0, 0.0, -1.0, 0.5, 1.0)], b3=(0.0, 0.0, 0.1))
    X = np.zeros((1, 32), np.float32)
    X[0, :3] = [1 + 2 ** -9, 1.0, 0.75]
    Y, H1, H2 = oracle.mlp_forward(B, X)
    assert H1[0, :3].tolist() == [1.0, 1 + 2 ** -7, 0.75]
    assert H2[0, :3].tolist() == [1.0, 1 + 2 ** -7, 0.0]
    assert Y[0].tolist() == [1.0, 1 + 2 ** -7, float(np.float32(0.1))]
    # the exact mode rounds nothing
    Ye, _, _ = oracle.mlp_forward(A, np.eye(1, 32, dtype=np.float32), exact=True)
    w = float(np.float32(1 + 2 ** -9))
    # (w2 = 1): y0 = w3 (w1 + b1 + b2) + b3
    assert abs(Ye[0, 0] - (w * (w + 6 * 2 ** -10) + float(np.float32(2 ** -12 + 2 ** -21)))) < 1e-12


def test_bf16_mode_tracks_the_exact_gradient():
    P = oracle.mlp_init(5)
    X, T = _batch(256, 6)
    _, Ge, _ = oracle.mlp_loss_grad(P, X, T, exact=True)
    _, Gb, _ = oracle.mlp_loss_grad(P, X, T, exact=False)
    cos = Ge @ Gb / np.linalg.norm(Ge) / np.linalg.norm(Gb)
    assert cos > 0.999


def test_adam_first_step_and_convergence():
    # first step of Adam is lr * g / (|g| + eps') in each coordinate
    P = np.array([1.0, -2.0, 0.5] + [0.0] * (oracle.MLP_NPARAM - 3), np.float32)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    g = np.zeros_like(P)
    g[:3] = [0.3, -4.0, 1e-3]
    P0 = P.copy()
    oracle.adam(P, g, m, v, 1, lr=1e-2, eps=1e-8)
    assert np.allclose(P[:3] - P0[:3], -1e-2 * np.sign(g[:3]), rtol=1e-4)
    assert (P[3:] == 0).all()
    # on f(p) = 0.5 * |p - p*|^2 Adam reaches the minimiser
    target = np.linspace(-1, 1, oracle.MLP_NPARAM).astype(np.float32)
    P = np.zeros(oracle.MLP_NPARAM, np.float32)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    for t in range(1, 3001):
        oracle.adam(P, P - target, m, v, t, lr=1e-2)
    assert np.abs(P - target).max() < 1e-2


def test_features_hand_built():
    img = np.full((64, 64), 100, np.uint8)
    ids = np.array([0, 1, 2, 3])
    xy = np.array([[30, 30], [33, 30], [30, 36], [50, 50]], np.float32)
    pxy = xy - np.array([[1, 2], [-16, 8], [0.5, 0.25], [3, 3]], np.float32)
    age = np.array([1, 1, 0, 2])
    F = oracle.features(ids, xy, pxy, age, img)
    # keypoint 0: tracks with a flow by distance: itself (0), 1 (d^2 = 9), 3 (800); 2 has age 0
    assert np.allclose(F[0, :6], [1 / 16, 2 / 16, -1.0, 0.5, 3 / 16, 3 / 16])
    assert (F[0, 6:16] == 0).all()
    # uniform image: every pooled cell equals the patch mean
    assert (F[:, 16:] == 0).all()
    # keypoint 2 (age 0, no flow of its own) gets its neighbours' flows: 0 (d^2 = 36), 1 (45), 3
    assert np.allclose(F[2, :6], [1 / 16, 2 / 16, -1.0, 0.5, 3 / 16, 3 / 16])
    # ties in distance go to the smaller id
    xy_t = np.array([[10, 10], [13, 10], [7, 10]], np.float32)
    F_t = oracle.features([5, 9, 2], xy_t, xy_t - 1, [0, 1, 1], img)
    assert np.allclose(F_t[0, :4], [1 / 16] * 4)  # ids 2 then 9, both at d^2 = 9
    # a bright left half: cells in the two left columns of the patch are brighter
    img2 = img.copy()
    img2[:, :30] = 200
    F2 = oracle.features(ids[:1], xy[:1], pxy[:1], age[:1], img2)
    cells = F2[0, 16:].reshape(4, 4)
    total = 8 * 16 * 200 + 8 * 16 * 100          # patch columns 22..37: 8 bright, 8 dark
    assert np.allclose(cells[:, :2], 200 * 16 * 16 / total - 1)
    assert np.allclose(cells[:, 2:], 100 * 16 * 16 / total - 1)


def test_learned_frontend_reduces_to_plain_and_to_the_small_budget():
    import synthgen
    w = synthgen.WORKLOADS["mono320"]
    seq = synthgen.sequence(w)
    P = np.zeros(oracle.MLP_NPARAM, np.float32)  # guess = 0 displacement
    recs = {}
    for name, mode, rho in (("plain", 0, 0.0), ("always_fallback", 1, -1.0), ("never_fallback", 1, 1e9)):
        fe = oracle.Frontend([w.width], [w.height], False,
                             oracle.params_for(w, init_mode=mode, learned_levels=2, learned_iters=3,
                                               learned_rho=rho))
        if mode:
            fe.set_mlp(P)
        fe.push([seq.frames[0, 0]])
        ids, xy, pxy, age = fe.keypoints(0)
        fe.push([seq.frames[1, 0]])
        recs[name] = (fe.records(), fe.last_fallback, xy)
        fe.close()
    a, b = recs["plain"][0], recs["always_fallback"][0]
    assert a.tobytes() == b.tobytes() and recs["always_fallback"][1] == len(recs["plain"][2])
    # rho = inf: a track kept by the 2-level, 3-iteration tracker from p (guess
    # 0) stays; the others fall back to the plain tracker (3 levels, 5 its)
    r, n_fb, xy = recs["never_fallback"]
    small, st_s = oracle.track(seq.frames[0, 0], seq.frames[1, 0], xy, xy, 2, 3)
    plain, st_p = oracle.track(seq.frames[0, 0], seq.frames[1, 0], xy, xy, w.levels, w.gn_iters)
    kept = st_s == oracle.TRACKED
    temporal = r[: len(xy)]
    assert n_fb == int((~kept).sum())
    assert (temporal["status"] == np.where(kept, st_s, st_p)).all()
    want_x = np.where(kept, small[:, 0], plain[:, 0])
    ok = temporal["status"] == oracle.TRACKED
    assert ok.sum() > 0.9 * len(xy)
    assert np.allclose(temporal["x"][ok], want_x[ok], atol=1e-5)
