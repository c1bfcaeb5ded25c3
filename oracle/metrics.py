"""Oracle of the map-quality metrics (Sec. V-C, Eq. 7, Eq. 8) -- TEST INFRASTRUCTURE ONLY.

The vertices of the reconstructed mesh form a point cloud M (with the vertices' labels),
compared with a ground-truth point cloud G (with its points' classes):

* d(p, G) = min(2 nu, |p - q|), q the point of G nearest to p (Eq. 7);
* RE = sqrt(mean over M of d(p, G)^2)                                   (Eq. 7);
* CD = mean over M of d(p, G) / 2 + mean over G of d(q, M) / 2           (Eq. 8);
* RC = the fraction of G with a point of M within 2 nu;
* mIoU and Acc (the semantic scores the paper takes from the SemanticKITTI benchmark),
  read here as: every ground-truth point with a vertex within 2 nu is evaluated, its
  predicted class being the label of its nearest vertex (an unlabelled vertex, 255, is a
  wrong prediction of no class); per class c, TP, FP and FN count evaluated points;
  IoU_c = TP / (TP + FP + FN) over the classes that occur; mIoU is their mean and Acc the
  fraction of evaluated points predicted correctly.

Nearest neighbours are exact (a k-d tree over float64 coordinates; ties go to the lower
index).  Everything here is float64.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def nearest(src, dst):
    """For each point of src its nearest point of dst: (distance, index); the lower index
    among equidistant points."""
    src = np.asarray(src, np.float64).reshape(-1, 3)
    dst = np.asarray(dst, np.float64).reshape(-1, 3)
    if len(dst) == 0:
        return np.full(len(src), np.inf), np.full(len(src), -1, np.int64)
    tree = cKDTree(dst)
    k = min(8, len(dst))
    d, i = tree.query(src, k=k)
    if k == 1:
        return d, i.astype(np.int64)
    d = d.reshape(len(src), k)
    i = i.reshape(len(src), k)
    best = d[:, :1] == d            # those of the 8 nearest at the nearest distance
    i_tie = np.where(best, i, np.iinfo(np.int64).max).min(axis=1)
    return d[:, 0], i_tie.astype(np.int64)


def mesh_metrics(M, M_lab, G, G_lab, voxel, n_classes):
    """RE, CD, RC, mIoU, Acc of the vertex cloud M (labels M_lab) against G (classes G_lab)."""
    cap = 2.0 * float(voxel)
    dM, _ = nearest(M, G)
    dG, iG = nearest(G, M)
    dpg = np.minimum(cap, dM)
    dqm = np.minimum(cap, dG)
    nM, nG = len(dM), len(dG)
    re = float(np.sqrt(np.mean(dpg ** 2))) if nM else 0.0
    cd = (0.5 * float(np.mean(dpg)) if nM else 0.0) + (0.5 * float(np.mean(dqm)) if nG else 0.0)
    covered = dG <= cap
    rc = float(np.mean(covered)) if nG else 0.0
    gt = np.asarray(G_lab, np.int64)[covered]
    pred = np.asarray(M_lab, np.int64)[iG[covered]] if nG else np.zeros(0, np.int64)
    conf = np.zeros((n_classes + 1, n_classes), np.int64)   # [pred (L = none)][gt]
    ok_gt = gt < n_classes
    p = np.where(pred < n_classes, pred, n_classes)
    np.add.at(conf, (p[ok_gt], gt[ok_gt]), 1)
    tp = np.diag(conf[:n_classes])
    fp = conf[:n_classes].sum(axis=1) - tp
    fn = conf.sum(axis=0) - tp
    occ = (tp + fp + fn) > 0
    miou = float(np.mean(tp[occ] / (tp + fp + fn)[occ])) if occ.any() else 0.0
    n_eval = int(ok_gt.sum())
    acc = float(tp.sum() / n_eval) if n_eval else 0.0
    return {"re": re, "cd": cd, "rc": rc, "miou": miou, "acc": acc, "n_eval": n_eval,
            "confusion": conf, "d_mg": dM, "d_gm": dG, "nn_gm": iG}
