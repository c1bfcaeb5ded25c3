"""Pins of the oracle's two other label-fusion modes (Sec. IV-C.3, Eq. 6; Sec. V-C):

* Eq. 6 taken literally, on per-pixel class log-probability images: checked against the
  vote counts (already pinned) through the textbook equivalence of a symmetric hard-label
  likelihood (log-posterior ratio = (n_l - n_max) log(p (L - 1) / (1 - p))), against a
  constant image's closed form, and against an fp64 recursive Bayes filter over a sequence
  of random distributions;
* Ours-wo-Bay, the latest label wins: checked against which calls saw each voxel.

Visibility (which voxels a camera updates, and at which pixel) is the counting mode's,
pinned in the label tests; these pins fix what each mode does with it.
"""
import numpy as np
import pytest

import oracle
import synth


def _maps(w, modes):
    out = []
    for mode in modes:
        om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, w.max_blocks)
        assert om.set_label_fusion(mode) == oracle.OK
        out.append(om)
    return out


def _frames(w, n):
    return [w.frame(k) for k in range(n)]


@pytest.fixture(scope="module")
def tiny():
    w = synth.tiny_workload()
    return w, _frames(w, 1)


def test_bayes_with_hard_label_likelihood_matches_counts(tiny):
    """Log-probabilities of a symmetric likelihood p for the observed class: the
    log-posterior of class l relative to the best is (n_l - n_max) log(p (L-1)/(1-p)) and
    the most probable class is the counts' argmax (Eq. 6 with hard labels)."""
    w, frames = tiny
    p = 0.7
    counts, bayes = _maps(w, (oracle.LABELS_COUNTS, oracle.LABELS_BAYES))
    L = w.n_classes
    f = frames[0]
    T_wc, lab, cam = f.cams[0]
    for om in (counts, bayes):
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    # three calls with the frame's label image and two shifted copies (different votes)
    imgs = [lab, np.roll(lab, 7, axis=1), np.roll(lab, -5, axis=0)]
    for im in imgs:
        assert counts.integrate_labels(cam, im, T_wc) == oracle.OK
        assert bayes.integrate_logprobs(cam, synth.hard_logprob_image(im, L, p), T_wc) == oracle.OK
    step = np.log(p * (L - 1) / (1 - p))
    n_checked = 0
    for b in counts.block_coords():
        c = counts.block(b)
        B = bayes.block(b)
        LP = bayes.block_logpost(b)
        n = c["counts"].astype(np.int64)            # [L, 512]
        seen = B["fused"] != 255
        nvis = (n.sum(axis=0) > 0)
        # every voxel with a vote was seen by the Bayes map, with the same number of calls
        assert np.all(seen[nvis])
        nmax = n.max(axis=0)
        unique = (n == nmax).sum(axis=0) == 1
        m = nvis & unique
        np.testing.assert_array_equal(B["fused"][m], c["fused"][m])
        want = (n - nmax)[:, m] * step
        assert np.all(np.abs(LP[:, m] - want) <= 1e-5 * (1 + np.abs(want)) * 3)
        n_checked += int(m.sum())
    assert n_checked > 10000


def test_bayes_constant_image_closed_form(tiny):
    """A constant distribution O seen n times: log-posterior n (log O_l - log O_max)."""
    w, frames = tiny
    L = w.n_classes
    rng = np.random.default_rng(3)
    logO = np.log(rng.dirichlet(np.ones(L))).astype(np.float32)
    counts, bayes = _maps(w, (oracle.LABELS_COUNTS, oracle.LABELS_BAYES))
    f = frames[0]
    T_wc, lab, cam = f.cams[0]
    for om in (counts, bayes):
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    const_lab = np.zeros_like(lab)
    img = np.broadcast_to(logO, (cam.height, cam.width, L)).copy()
    for _ in range(3):
        counts.integrate_labels(cam, const_lab, T_wc)
        bayes.integrate_logprobs(cam, img, T_wc)
    best = int(np.argmax(logO))
    ratio = logO.astype(np.float64) - logO.astype(np.float64).max()
    n_vis = 0
    for b in counts.block_coords():
        n = counts.block(b)["counts"][0].astype(np.int64)
        B = bayes.block(b)
        LP = bayes.block_logpost(b)
        vis = n > 0
        assert np.all(B["fused"][vis] == best) and np.all(B["fused"][~vis] == 255)
        want = n[vis][None, :] * ratio[:, None]
        assert np.all(np.abs(LP[:, vis] - want) <= 1e-5 * (1 + np.abs(want)) * 4)
        assert not np.any(LP[:, ~vis])
        n_vis += int(vis.sum())
    assert n_vis > 10000


def test_bayes_matches_fp64_recursive_filter():
    """A voxel-independent check: one block set by a frame, then five random distribution
    images; every visible voxel's posterior equals an fp64 recursive Bayes filter (Eq. 6,
    P <- P O / Z) run over the same pixels' distributions, the pixels being the ones the
    counting mode votes at (a pixel-encoding label image gives them)."""
    w = synth.tiny_workload()
    f = w.frame(0)
    T_wc, lab, cam = f.cams[0]
    L = w.n_classes
    counts_maps = []
    bayes, = _maps(w, (oracle.LABELS_BAYES,))
    assert bayes.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    # which pixel each voxel reads: counting maps with label images that encode the
    # pixel's column and row as base-L digits (three each: L^3 > 640)
    H, W_ = cam.height, cam.width
    uu, vv = np.meshgrid(np.arange(W_), np.arange(H))
    codes = [(x // L ** d) % L for x in (uu, vv) for d in range(3)]
    for code in codes:
        om, = _maps(w, (oracle.LABELS_COUNTS,))
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
        assert om.integrate_labels(cam, code.astype(np.uint8), T_wc) == oracle.OK
        counts_maps.append(om)
    rng = np.random.default_rng(11)
    imgs = [np.log(rng.dirichlet(np.ones(L) * 0.7, size=(H, W_))).astype(np.float32) for _ in range(5)]
    for im in imgs:
        assert bayes.integrate_logprobs(cam, im, T_wc) == oracle.OK
    stack = np.stack(imgs).astype(np.float64)        # [5, H, W, L]
    n_checked = 0
    for b in bayes.block_coords():
        B = bayes.block(b)
        vis = B["fused"] != 255
        if not vis.any():
            continue
        digits = [cm.block(b)["fused"].astype(np.int64) for cm in counts_maps]
        u = digits[0] + L * digits[1] + L * L * digits[2]
        v = digits[3] + L * digits[4] + L * L * digits[5]
        idx = np.nonzero(vis)[0]
        logpost = stack[:, v[idx], u[idx], :].sum(axis=0)      # [n, L] fp64
        logpost -= logpost.max(axis=1, keepdims=True)
        LP = bayes.block_logpost(b)[:, idx].T
        assert np.all(np.abs(LP - logpost) <= 2e-5 * (1 + np.abs(logpost)))
        top2 = np.sort(logpost, axis=1)[:, -2]
        clear = top2 < -1e-3
        np.testing.assert_array_equal(B["fused"][idx][clear], np.argmax(logpost, axis=1)[clear])
        n_checked += len(idx)
    assert n_checked > 10000


def test_latest_label_wins(tiny):
    """Ours-wo-Bay: a voxel takes the label of its latest observation; the calls' order
    decides, counts stay untouched."""
    w, frames = tiny
    f = frames[0]
    T_wc, lab, cam = f.cams[0]
    latest, first_only = _maps(w, (oracle.LABELS_LATEST, oracle.LABELS_COUNTS))
    for om in (latest, first_only):
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    a = np.full_like(lab, 3)
    b_img = np.full_like(lab, 5)
    b_img[:, : cam.width // 2] = 255     # the second call labels only the right half
    assert latest.integrate_labels(cam, a, T_wc) == oracle.OK
    assert latest.integrate_labels(cam, b_img, T_wc) == oracle.OK
    assert first_only.integrate_labels(cam, b_img, T_wc) == oracle.OK   # who the second call reached
    n3 = n5 = 0
    for blk in latest.block_coords():
        L_ = latest.block(blk)
        C = first_only.block(blk)
        second = C["counts"][5] > 0
        assert np.all(L_["fused"][second] == 5)
        rest = L_["fused"][~second]
        assert np.all((rest == 3) | (rest == 255))
        assert not np.any(L_["counts"])
        n3 += int((rest == 3).sum())
        n5 += int(second.sum())
    assert n3 > 1000 and n5 > 1000
    assert latest.stats()["votes"] > n5


def test_modes_reject_the_other_input(tiny):
    w, frames = tiny
    f = frames[0]
    T_wc, lab, cam = f.cams[0]
    counts, bayes = _maps(w, (oracle.LABELS_COUNTS, oracle.LABELS_BAYES))
    for om in (counts, bayes):
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    assert bayes.integrate_labels(cam, lab, T_wc) == oracle.INVALID
    assert counts.integrate_logprobs(cam, synth.hard_logprob_image(lab, w.n_classes, 0.7), T_wc) == oracle.INVALID
    assert counts.set_label_fusion(3) == oracle.INVALID
