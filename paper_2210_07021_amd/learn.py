"""Training of the per-interaction order network (the learned order policy).

The labels come from the FP64 sFMM itself (sfmm_order_samples: the exact
smallest order per sampled FMM act for the tolerance), the network is
trained on the GPU by the library's own kernels (sfmm_mlp_train), and a plan
uses it with order_policy=SFMM_ORDER_LEARNED, mlp_weights=weights.
"""
from __future__ import annotations

import numpy as np


def order_training_data(skies_, tolerance: float, leaf_size: int = 32, samples_per_sky: int = 60000,
                        seed: int = 0):
    """Features [n][8] and labels [n] (in orders) from the given skies,
    each a (src, q, tgt) triple: the FP64 plan at the tolerance is executed
    and samples_per_sky of its FMM acts are labelled."""
    import torch
    from . import Plan
    fs, ls = [], []
    for i, (src, q, tgt) in enumerate(skies_):
        plan = Plan(src, q, tgt, tolerance=tolerance, leaf_size=leaf_size)
        plan.execute()
        torch.cuda.synchronize()
        f, l = plan.order_samples(samples_per_sky, seed=seed + i)
        plan.close()
        fs.append(f)
        ls.append(l)
    return np.concatenate(fs), np.concatenate(ls)


def train_order_network(features, labels, epochs: int = 30, batch: int = 512, lr: float = 1e-3, seed: int = 0):
    """Trains the network on (features, labels in orders); returns (weights,
    loss per epoch).  The network predicts (order - 16) / 8."""
    from . import mlp_init, mlp_train
    w0 = mlp_init(seed)
    return mlp_train(features, (np.asarray(labels, np.float32) - 16.0) / 8.0, w0, epochs=epochs, batch=batch,
                     lr=lr, seed=seed)
