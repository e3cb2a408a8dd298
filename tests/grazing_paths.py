"""Straight particle paths that cross an element face at grazing incidence.

Test-side construction: a random point on a random internal face (through the
oracle's element map), a direction at angle phi to the face's tangent plane
(phi log-uniform), and a start point a fraction of one step length behind the
face point.  Used to pin the tracking where the face intersection is
ill-conditioned (root error ~ 1/sin(phi)) on both codes.
"""
import numpy as np


def grazing_paths(o, mesh, n, rng, step_len, log_phi=(-7.0, -1.0)):
    x0s, ds, hints = [], [], []
    while len(x0s) < n:
        e = int(rng.integers(mesh.n_elem))
        f = int(rng.integers(6))
        if mesh.nbr_elem[e, f] < 0 or mesh.bc[e, f] != 0:
            continue
        ax = f // 2
        free = [a for a in range(3) if a != ax]
        xi = np.zeros(3)
        xi[ax] = 1.0 if f % 2 else -1.0
        xi[free[0]], xi[free[1]] = rng.uniform(-0.9, 0.9, 2)
        x, J = o.map(e, xi)
        t1, t2 = J[:, free[0]], J[:, free[1]]
        nrm = np.cross(t1, t2)
        nrm /= np.linalg.norm(nrm)
        if np.dot(nrm, J[:, ax]) * (1.0 if f % 2 else -1.0) < 0:
            nrm = -nrm                                  # outward normal of e
        th = rng.uniform(0.0, 2.0 * np.pi)
        tg = np.cos(th) * t1 / np.linalg.norm(t1) + np.sin(th) * t2 / np.linalg.norm(t2)
        tg -= np.dot(tg, nrm) * nrm
        tg /= np.linalg.norm(tg)
        phi = 10.0 ** rng.uniform(*log_phi)
        d = np.cos(phi) * tg + np.sin(phi) * nrm
        x0s.append(x - d * step_len * rng.uniform(0.2, 0.8))
        ds.append(d)
        hints.append(e)
    return np.array(x0s), np.array(ds), np.array(hints, np.int32)
