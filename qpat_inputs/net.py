"""Seeded initial weights of the learned-guess network (random draws only).

He-normal weights w ~ N(0, 2 / (27 c_in)), zero biases, flattened layer by
layer as w[c_out][c_in][27] then b[c_out] (stream 5 of the workload's seed).
"""
import numpy as np

from .configs import rng

NET_CHANNELS = (3, 16, 16, 16, 1)


def initial_params(cfg_id):
    g = rng(cfg_id, 5)
    out = []
    for cin, cout in zip(NET_CHANNELS[:-1], NET_CHANNELS[1:]):
        out.append(g.standard_normal(cout * cin * 27) * np.sqrt(2.0 / (27 * cin)))
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32)
