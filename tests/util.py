"""Shared test helpers: problem set-ups built from the seeded input generators."""
import numpy as np

import oracle as O
from paper_2205_07824_amd import inputs as I


def penalty(p, h):
    """Interior-penalty parameter tau = (p+1)^2 / h (reading settled by the MMS-rate pin)."""
    return (p + 1) ** 2 / h


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def poisson_setup(nd, n, p, mms, nq=None, perturb=0.0, seed=0, kappa=1.0, lam=0.0):
    box = I.box_mesh(nd, n, perturb=perturb, seed=seed)
    m = O.Mesh(box, p, nq)
    xn, xq, xb, bf = m.points()
    _, _, f = mms(xq)
    ub, _, _ = mms(xb)
    tau = penalty(p, 1.0 / n)
    md = O.Model(O.MODEL_POISSON, 1, [kappa, tau, lam], src=f.reshape(m.E, 1, m.nqv),
                 bdata=ub.reshape(m.nbf, 1, m.nqf), bc_kind=[0])
    return box, m, md
