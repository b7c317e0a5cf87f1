"""Seeded request streams for the serving loop (Poisson arrivals).

Each request applies V_X (op 0) or K_ACE (op 1) to a block of `block`
consecutive orbitals of one trajectory, at a uniformly drawn block index.
Trajectories are drawn by class with the given mix; inter-arrival times are
exponential with the given mean rate.
"""
from __future__ import annotations

import numpy as np


def poisson_requests(seed, n_requests, rate_per_s, trajs_by_class, class_mix, block=8, vx_share=0.5):
    """trajs_by_class: {class: [(traj_id, n_orbitals), ...]}; class_mix: {class: probability}.

    Returns a list of dicts(traj, op, first, count, t) sorted by arrival time t (seconds).
    """
    rng = np.random.default_rng(seed)
    classes = sorted(class_mix)
    probs = np.array([class_mix[c] for c in classes], dtype=float)
    probs /= probs.sum()
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        c = classes[rng.choice(len(classes), p=probs)]
        traj, n = trajs_by_class[c][rng.integers(len(trajs_by_class[c]))]
        count = min(block, n)
        nblocks = max(1, n // count)
        first = int(rng.integers(nblocks)) * count
        op = 0 if rng.random() < vx_share else 1
        out.append(dict(traj=int(traj), op=op, first=first, count=count, t=t))
    return out
