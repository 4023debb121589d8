"""Run independent oracle derivatives in parallel host processes (test helper).

Each complex-step derivative through a load path is one independent oracle
run; the GPU tests evaluate dozens of them, so they are spread over a pool of
fresh interpreter processes (spawned, so nothing of the caller's GPU context
is inherited) with single-threaded BLAS.
"""
import multiprocessing as mp
import os


def _init():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"


def _path_derivative(args):
    from oracle.adjoint import path_directional_derivative
    kw = args.pop("kw", {})
    return path_directional_derivative(**args, **kw)


def path_derivatives(K, w, alpha, beta, fiber, matrix, E, g, directions, workers=None,
                     compressed=False):
    """Complex-step path derivatives dJ/dtheta . v for every (v_w, v_alpha, v_beta)
    in directions, computed in parallel; returns a list in the same order."""
    jobs = [dict(K=K, w=w, alpha=alpha, beta=beta, fiber=fiber, matrix=matrix, E_paths=E,
                 g=g, v_w=vw, v_alpha=va, v_beta=vb, kw=dict(compressed=compressed))
            for vw, va, vb in directions]
    workers = workers or min(16, os.cpu_count() or 1, len(jobs))
    if workers <= 1:
        return [_path_derivative(j) for j in jobs]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_init) as pool:
        return pool.map(_path_derivative, jobs, chunksize=1)


def unit_directions(K, w_idx, a_idx):
    """Unit directions for the selected weights, then alphas, then betas."""
    import numpy as np
    nl, L = 2 ** K, 2 ** K - 1
    out = []
    for j in w_idx:
        vw = np.zeros(nl)
        vw[j] = 1.0
        out.append((vw, np.zeros(L), np.zeros(L)))
    for which in (1, 2):
        for p in a_idx:
            v = [np.zeros(nl), np.zeros(L), np.zeros(L)]
            v[which][p] = 1.0
            out.append(tuple(v))
    return out
