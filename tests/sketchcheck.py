"""Comparison of a device array with a stored oracle sketch (norm and
separable random projections, see workloads.sketch).  The projections are
contracted on the device in FP64 (rounding ~1e-14 of the norm)."""

import numpy as np

import workloads


def device_sketch(X, nproj):
    import torch
    out = []
    for k in range(nproj):
        vs = workloads.sketch_vectors(tuple(X.shape), k)
        Y = X
        for ax in range(X.dim() - 1, -1, -1):
            Y = Y @ torch.from_numpy(vs[ax]).to(X.device)
        out.append(float(Y))
    return np.asarray(out)


def sketch_error(X, entry):
    """(estimated relative l2 error over the whole array, relative norm
    difference) of device array X against the stored entry."""
    import torch
    ref = np.asarray(entry["sketch"])
    got = device_sketch(X, ref.size)
    nrm = entry["norm"]
    est = float(np.sqrt(np.mean((got - ref) ** 2)) / nrm)
    dn = abs(float(torch.linalg.vector_norm(X)) - nrm) / nrm
    return est, dn
