"""GPU learned-initialisation part against the CPU oracle, through the C ABI.

Network forward and gradient: the oracle emulates the GPU's bfloat16 rounding
points; the remaining difference is the MFMA's summation order inside a
32-wide step (a rare 1-ulp flip of a bf16 activation). Features: bit-exact.
Learned pipeline: records parity with state injection.
"""
import numpy as np
import pytest

import oracle
import synthgen
from parity_util import Tally, _track_fp64, compare_records, inject, oracle_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 0.5, (n, 32)).astype(np.float32)
    T = rng.normal(0, 2.0, (n, 2)).astype(np.float32)
    return X, T


@pytest.mark.parametrize("n", [1, 16, 37, 600, 1000])
def test_forward_matches_oracle(n):
    import torch
    import paper_2609_30459_amd as vf
    P = oracle.mlp_init(7)
    P[-3:] = [0.05, -0.02, 0.1]
    X, _ = _data(n, n)
    want, _, _ = oracle.mlp_forward(P, X)
    with vf.Mlp(1024) as net:
        net.set_params(P)
        y = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
        net.forward(torch.from_numpy(X).cuda(), y)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
    scale = np.abs(want).mean() + 1e-3
    assert np.abs(got - want).max() <= 2e-2 * scale, (np.abs(got - want).max(), scale)
    assert np.median(np.abs(got - want)) <= 1e-3 * scale


def _term_magnitudes(P, X, T):
    """A[p] = sum over the batch of |a| |b| for the two operands of every
    weight-gradient product (dW = dH^T H_prev, db = sum dH): the most that
    one-ulp bfloat16 differences in all operands can move dW is 2^-8 A for
    each operand. Built from the oracle's forward and loss; the backward
    operands are propagated here only to size the tolerance."""
    bf = np.vectorize(oracle.bf16, otypes=[np.float32])
    Y, H1, H2 = oracle.mlp_forward(P, X)
    _, _, dY = oracle.mlp_loss_grad(P, X, T)
    W2 = bf(P[4224:20608].reshape(128, 128)).astype(np.float64)
    W3 = bf(P[20736:21120].reshape(3, 128)).astype(np.float64)
    dH2 = np.abs(dY) @ np.abs(W3) * (H2 > 0)
    dH1 = dH2 @ np.abs(W2) * (H1 > 0)
    Xb = np.abs(bf(X).astype(np.float64))
    A = np.zeros(oracle.MLP_NPARAM)
    A[0:4096] = (dH1.T @ Xb).ravel()
    A[4096:4224] = dH1.sum(0)
    A[4224:20608] = (dH2.T @ np.abs(H1)).ravel()
    A[20608:20736] = dH2.sum(0)
    A[20736:21120] = (np.abs(dY).T @ np.abs(H2)).ravel()
    A[21120:21123] = np.abs(dY).sum(0)
    return A


@pytest.mark.parametrize("n", [32, 300, 1024])
def test_gradient_matches_oracle(n):
    """dW element by element: within 1e-2 of the oracle's value plus 2^-7 of
    the element's term magnitude (one-ulp bfloat16 differences of both
    operands, from the MFMA's summation order flipping a rounding)."""
    import torch
    import paper_2609_30459_amd as vf
    P = oracle.mlp_init(9)
    X, T = _data(n, 100 + n)
    L_o, G_o, _ = oracle.mlp_loss_grad(P, X, T)
    with vf.Mlp(1024) as net:
        net.set_params(P)
        g = torch.zeros(vf.MLP_NPARAM, dtype=torch.float32, device="cuda")
        L_g = net.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), g)
        G_g = g.cpu().numpy().astype(np.float64)
    assert abs(L_g - L_o) <= 1e-3 * abs(L_o)
    A = _term_magnitudes(P, X, T)
    err = np.abs(G_g - G_o)
    tol = 1e-2 * np.abs(G_o) + 2.0 ** -7 * A
    bad = np.nonzero(err > tol)[0]
    assert not len(bad), (f"{len(bad)} gradient entries outside tolerance, first {bad[:5].tolist()}: "
                          f"gpu {G_g[bad[:5]].tolist()} oracle {G_o[bad[:5]].tolist()} A {A[bad[:5]].tolist()}")
    # most entries agree far inside the bound (a flip is rare)
    rel = err / np.maximum(np.abs(G_o), 1e-30)
    assert np.median(rel[np.abs(G_o) > 1e-6]) < 1e-4


def test_adam_step_matches_oracle_and_training_reduces_loss():
    """The GPU's Adam step against the oracle's Adam applied to the GPU's own
    gradient of the same batch (the gradient kernels are deterministic): each
    weight's move within 1e-2 of the expected move (first and second step;
    a wrong learning rate, epsilon or bias correction fails)."""
    import torch
    import paper_2609_30459_amd as vf
    P = oracle.mlp_init(11)
    X, T = _data(1024, 5)
    with vf.Mlp(1024) as net:
        net.set_params(P)
        dx, dt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
        g = torch.zeros(vf.MLP_NPARAM, dtype=torch.float32, device="cuda")
        P_o, m, v = P.copy(), np.zeros_like(P), np.zeros_like(P)
        for step in (1, 2):
            before = net.get_params()
            net.gradient(dx, dt, g)
            G = g.cpu().numpy()
            oracle.adam(P_o, G, m, v, step, lr=1e-3)
            loss = net.train_step(dx, dt, lr=1e-3)
            P_g = net.get_params()
            want = P_o.astype(np.float64) - before
            got = P_g.astype(np.float64) - before
            # float rounding of the parameter itself: 2 ulps of |P|
            tol = 1e-2 * np.abs(want) + 2.0 ** -22 * np.abs(before)
            bad = np.nonzero(np.abs(got - want) > tol)[0]
            assert not len(bad), (step, len(bad), got[bad[:5]].tolist(), want[bad[:5]].tolist())
            assert np.median(np.abs(want)) > 5e-4  # the steps are about lr in size
            P_o = P_g.copy()  # the next step starts from the GPU's parameters
            if step == 1:
                loss0 = loss
        losses = [net.train_step(dx, dt, lr=1e-3) for _ in range(200)]
    assert losses[-1] < 0.5 * loss0


def _learned_params(w, rho, levels=2, iters=3):
    return dict(init_mode=1, learned_levels=levels, learned_iters=iters, learned_rho=rho)


def _learned_run(w, seq, P, rho, launch, frames, where, extra=None, k=1):
    """Learned-init GPU frontend against the oracle with state injection: records,
    features (bit-exact) and fallback counts (exact) per frame; returns the
    total fallbacks. extra: further parameters for both sides; k: the
    keypoints per cell, whose referral cap the run's tally is held to. The
    FP64 referee rebuilds the starts it knows: every record of the first frame,
    the stereo matches from the disparity prior and, when every learned track
    falls back (rho < 0) with the full budget, the temporal tracks (constant-
    velocity start); any other record outside the tolerance fails."""
    import paper_2609_30459_amd as vf
    po = {**_learned_params(w, rho), **(extra or {})}
    fe_o = oracle.Frontend([w.width] * w.n_cams, [w.height] * w.n_cams, w.stereo, oracle.params_for(w, **po))
    fe_o.set_mlp(P)
    n_fb = 0
    tally = Tally(where)
    with vf.Frontend([(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size)],
                     vf.params_for(w, **po, **launch)) as fe_g:
        fe_g.set_mlp(P)
        for t in range(frames):
            if t > 0:
                inject(fe_g, fe_o, 0, w.n_cams)
                state = [fe_o.keypoints(c) for c in range(w.n_cams)]
            prev = [oracle_state(fe_o, c) for c in range(w.n_cams)]
            fe_o.push(list(seq.frames[t]))
            fe_g.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            g, o = fe_g.get_tracks(0), fe_o.records()

            def referee(idx, t=t, o=o, prev=prev):
                all_fall_back = rho < 0 and not po.get("learned_fb_levels", 0)
                learned_start = (o["status"][idx] == oracle.TRACKED) & (t > 0) & (not all_fall_back)
                if po.get("stereo_init", 0) != 0 and t > 0:
                    learned_start |= o["status"][idx] == oracle.MATCHED
                assert not learned_start.any(), f"{where} frame {t}: a learned-start record outside the tolerance"
                return _track_fp64(seq.frames, t, o, prev, idx, w.levels, w.gn_iters, w.fb_threshold, w.disparity0)

            compare_records(g, o, w.fb_threshold, where=f"{where} frame {t}", tally=tally,
                            referee=referee if k > 1 else None)
            if t > 0:
                for c in range(w.n_cams):
                    ids, xy, pxy, age = state[c]
                    want = oracle.features(ids, xy, pxy, age, seq.frames[t - 1, c])
                    got = fe_g.get_features(0, c)
                    assert got.shape == want.shape
                    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), c
                st = fe_g.stats()
                assert st["last_fallback"] == fe_o.last_fallback, (t, st["last_fallback"], fe_o.last_fallback)
                n_fb += st["last_fallback"]
    fe_o.close()
    print(tally.line(), f"fallbacks {n_fb}", flush=True)
    tally.check(k)
    return n_fb


FB25 = dict(learned_fb_levels=2, learned_fb_iters=5)
NB23 = dict(stereo_init=1, stereo_levels=2, stereo_iters=3)


@pytest.mark.parametrize("rho,launch,extra", [(-1.0, {}, {}), (0.02, {}, {}), (1e9, {}, {}), (0.02, {"eager": True}, {}),
                                              (0.02, {"stereo_mode": 1, "track_waves_per_cu": 4}, {}),
                                              (-1.0, {}, FB25), (0.02, {}, {**FB25, **NB23}),
                                              (0.02, {"stereo_mode": 1}, {**FB25, **NB23}),
                                              (0.02, {"learned_block_waves": 8}, {}),
                                              (-1.0, {"learned_block_waves": 16}, {**FB25, **NB23}),
                                              (0.02, {"learned_fused": 1}, {}),
                                              (-1.0, {"learned_fused": 1, "track_parallel_fallback": 1},
                                               {**FB25, **NB23}),
                                              (0.02, {"learned_fused": 1, "track_waves_per_cu": 4, "stereo_mode": 1},
                                               FB25)])
def test_learned_pipeline_parity_and_features(rho, launch, extra):
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=7, n_frames=4)
    P = oracle.mlp_init(13) * 0.05
    P[-3:] = 0.0
    n_fb = _learned_run(w, seq, P, rho, launch, 4, f"learned stereo752 rho={rho} {launch} {extra}", extra)
    if rho < 0:
        assert n_fb > 0


def test_learned_pipeline_parity_trained_weights_stereo1280():
    """The committed trained network on its own workload (1280x720 stereo, held-out
    sequence): the learned guesses, short budget and fallbacks as in the
    benchmark, against the oracle."""
    from paper_2609_30459_amd.train_mlp import load_weights
    import os
    import paper_2609_30459_amd as vf
    P, rho, _ = load_weights(os.path.join(os.path.dirname(vf.__file__), "weights", "mlp_stereo1280.bin"))
    w = synthgen.WORKLOADS["stereo1280"]
    seq = synthgen.sequence(w, seq=3, n_frames=5)
    n_fb = _learned_run(w, seq, P, rho, {}, 5, "learned stereo1280 trained weights")
    assert n_fb > 0  # the fallback path is exercised
    # the benchmark's learned configuration: 2 x 5 fallback, neighbour stereo start, with the learned stage
    # fused into the tracker and the fallbacks computed beside the short attempts
    n_fb = _learned_run(w, seq, P, rho, {"learned_fused": 1, "track_parallel_fallback": 1}, 5,
                        "learned stereo1280 trained weights, 2x5 fallback, neighbour stereo, fused", {**FB25, **NB23})
    assert n_fb > 0


@pytest.mark.parametrize("name,launch", [("stereo1280", {}), ("stereo1280", {"track_parallel_fallback": 1}),
                                         ("stereo752", {"stereo_mode": 1}),
                                         ("stereo752", {"track_waves_per_cu": 4, "track_block_waves": 2})])
def test_fused_learned_stage_equals_its_own_launch_bitwise(name, launch):
    """The learned stage fused into the tracker gives the records, features and
    fallback counts of its own launch, bit for bit (trained weights)."""
    from paper_2609_30459_amd.train_mlp import load_weights
    import os
    import paper_2609_30459_amd as vf
    P, rho, _ = load_weights(os.path.join(os.path.dirname(vf.__file__), "weights", "mlp_stereo1280.bin"))
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=6, n_frames=6)
    stream = (w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size)
    po = dict(_learned_params(w, rho), **FB25, **NB23)
    fbs = 0
    with vf.Frontend([stream], vf.params_for(w, **po, **launch)) as a, \
            vf.Frontend([stream], vf.params_for(w, learned_fused=1, **po, **launch)) as b:
        a.set_mlp(P, rho)
        b.set_mlp(P, rho)
        for t in range(6):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            ra, rb = a.get_tracks(0), b.get_tracks(0)
            assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), t
            sa, sb = a.stats(), b.stats()
            assert sa["last_fallback"] == sb["last_fallback"], t
            fbs += sa["last_fallback"]
            if t > 0:
                for c in range(w.n_cams):
                    assert a.get_features(0, c).tobytes() == b.get_features(0, c).tobytes(), (t, c)
    assert fbs > 0




@pytest.mark.parametrize("waves", [4, 16, 0])
def test_learned_features_span_several_staged_chunks(waves):
    """Eight keypoints per cell on 1280x720 (about 3000 live keypoints per
    camera): the learned stage stages the camera's tracks in LDS 2048 at a
    time, so the nearest-neighbour search crosses chunks; features bit-exact,
    exact fallback counts and records against the oracle (k > 1 bar) for two
    workgroup shapes and with the stage fused into the tracker (waves 0: each
    track's wave reads the tracks straight from global memory)."""
    import dataclasses
    w = dataclasses.replace(synthgen.WORKLOADS["stereo1280"], max_keypoints=3240, k_per_cell=8)
    seq = synthgen.sequence(w, seq=5, n_frames=3)
    P = oracle.mlp_init(17) * 0.05
    P[-3:] = 0.0
    fe_o = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
    try:
        fe_o.push(list(seq.frames[0]))
        n_live = min(len(fe_o.keypoints(c)[0]) for c in range(2))
    finally:
        fe_o.close()
    assert n_live > 2048, n_live
    # every learned track falls back, so the FP64 referee can rebuild every record
    launch = {"learned_fused": 1} if waves == 0 else {"learned_block_waves": waves}
    n_fb = _learned_run(w, seq, P, -1.0, launch, 3, f"learned k=8 {launch}", k=8)
    assert n_fb > 4000
