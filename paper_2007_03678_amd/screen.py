"""Host logic of a screened campaign: pick the ligands a pre-screen ranks
best, and judge the pick by plain docking.

Scores follow the docking convention (lower = better).  Everything numerical
on the GPU (prediction, training, docking) goes through the C ABI; this
module only sorts and counts.
"""
from __future__ import annotations

import math

import numpy as np


def top_fraction(scores, frac: float) -> np.ndarray:
    """Indices of the ceil(frac * n) lowest scores (ties by index)."""
    s = np.asarray(scores, dtype=np.float64)
    k = min(len(s), int(math.ceil(frac * len(s) - 1e-9)))
    return np.argsort(s, kind="stable")[:k]


def recall(judge_scores, selected, top_frac: float = 0.01):
    """(hits, positives): how many of the judge's top `top_frac` ligands
    (lowest judge scores) are among `selected`."""
    pos = set(top_fraction(judge_scores, top_frac).tolist())
    hits = len(pos & set(np.asarray(selected).tolist()))
    return hits, len(pos)


def clopper_pearson(k: int, n: int, alpha: float = 0.05):
    """Exact two-sided (1 - alpha) interval of a binomial proportion."""
    from scipy.stats import beta
    lo = 0.0 if k == 0 else float(beta.ppf(alpha / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - alpha / 2, k + 1, n - k))
    return lo, hi


def fraction_for_recall(pred_scores, judge_scores, target: float = 0.95, top_frac: float = 0.01) -> float:
    """Smallest fraction f such that the predicted top f holds at least
    `target` of the judge's top `top_frac`."""
    pred = np.asarray(pred_scores, dtype=np.float64)
    order = np.argsort(pred, kind="stable")
    rank = np.empty(len(order), dtype=np.int64)
    rank[order] = np.arange(len(order))
    pos = np.sort(rank[top_fraction(judge_scores, top_frac)])
    need = int(math.ceil(target * len(pos) - 1e-9))
    return float(pos[need - 1] + 1) / len(pred)


def average_rank(values) -> np.ndarray:
    """Ranks 1..n of `values` in ascending order, tied values sharing the
    mean of the ranks they span."""
    v = np.asarray(values, dtype=np.float64)
    order = np.argsort(v, kind="stable")
    sv = v[order]
    first = np.concatenate(([True], sv[1:] != sv[:-1]))
    group = np.cumsum(first) - 1                       # tie group of each sorted value
    start = np.flatnonzero(first)                      # first sorted position of each group
    end = np.concatenate((start[1:], [len(sv)]))       # one past its last
    out = np.empty(len(v), dtype=np.float64)
    out[order] = 0.5 * (start[group] + end[group] + 1)
    return out


def prior_score(pred_scores, n_atoms, weight: float) -> np.ndarray:
    """Ranking score of the screen (lower = better): the pre-screen's rank
    plus `weight` times the rank by ligand size, larger ligands first."""
    r = average_rank(pred_scores)
    if weight == 0:
        return r
    return r + weight * average_rank(-np.asarray(n_atoms, dtype=np.float64))


def choose_prior_weight(pred_scores, labels, n_atoms, target: float = 0.95, top_frac: float = 0.01,
                        weights=(0.0, 0.25, 0.5, 0.75, 1.0, 1.5, 2.0)):
    """(weight, share): the size-prior weight whose ranking of a validation
    set needs the smallest share of the list for `target` recall of the
    labels' top `top_frac` (the smaller weight on ties)."""
    best = None
    for w in weights:
        f = fraction_for_recall(prior_score(pred_scores, n_atoms, w), labels, target, top_frac)
        if best is None or f < best[1] - 1e-12:
            best = (float(w), f)
    return best
