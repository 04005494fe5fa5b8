"""Writes dip_64x64_degrees.txt: the per-cell degrees of the 2-D 64 x 64
workload whose obstacle has a dip (phi = 0.2 - 0.15 exp(-20 |x - x0|^2), data
seed 0), graded from p = 2 at the contact boundary to p = 12 far from it.

Recipe (calls only the oracle):
  1. pilot solve on the same mesh at uniform p = 2 (oracle LVPP loop, default
     options);
  2. contact cells: cell mean of exp(-psi_h) below 1e-6;
  3. contact boundary: the mesh edges between a contact and a non-contact cell;
  4. dist = Euclidean distance from each cell centre to the nearest point of
     that boundary;
  5. p_K = 2 if dist <= 0.1, 12 if dist >= 0.4, else round-half-up of
     2 + 10 (dist - 0.1) / 0.3.  An empty contact set gives p = 12 everywhere.
Output: 64 lines of 64 integers, line j = cells (0..63, j), direction 0 fastest.
Run: python tests/golden/make_dip_degrees.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from oracle import assemble, lvpp, mesh as OM   # noqa: E402
import workloads as W   # noqa: E402

M = 64


def main():
    f, phi = W.w2d_dip(0)
    br = W.uniform_breaks(M)
    mesh = OM.TensorMesh([br, br], 2)
    x = mesh.quadrature_points()
    sysm = assemble.System(mesh, f(x), phi(x))
    res = lvpp.solve(sysm, lvpp.Options())
    print("pilot: converged", res.converged, "prox", res.prox_steps, "newton", res.newton)
    pq = sysm.psi_at_points(res.psi)[:, 0, :]            # (cells, Q)
    W_ = np.array([c[2] for c in sysm.cells])            # quadrature weights |J| w
    mean = np.sum(W_ * np.exp(np.minimum(-pq, 700.0)), axis=1) / np.sum(W_, axis=1)
    contact = (mean < 1e-6).reshape(M, M)                # [j, i]: cell (i, j)
    h = 1.0 / M
    segs = []
    for j in range(M):
        for i in range(M):
            if i + 1 < M and contact[j, i] != contact[j, i + 1]:
                xe = (i + 1) * h
                segs.append(((xe, j * h), (xe, (j + 1) * h)))
            if j + 1 < M and contact[j, i] != contact[j + 1, i]:
                ye = (j + 1) * h
                segs.append(((i * h, ye), ((i + 1) * h, ye)))
    deg = np.full((M, M), 12, dtype=int)
    if not segs:
        print("empty contact set: p = 12 everywhere")
    else:
        a = np.array([s[0] for s in segs])
        b = np.array([s[1] for s in segs])
        for j in range(M):
            for i in range(M):
                c = np.array([(i + 0.5) * h, (j + 0.5) * h])
                ab = b - a
                t = np.clip(np.sum((c - a) * ab, axis=1) / np.sum(ab * ab, axis=1), 0.0, 1.0)
                dist = np.min(np.linalg.norm(a + t[:, None] * ab - c, axis=1))
                if dist <= 0.1:
                    deg[j, i] = 2
                elif dist >= 0.4:
                    deg[j, i] = 12
                else:
                    deg[j, i] = int(np.floor(2 + 10 * (dist - 0.1) / 0.3 + 0.5))
    print("contact cells", int(contact.sum()), "boundary edges", len(segs),
          "degree histogram", np.bincount(deg.reshape(-1), minlength=13)[2:].tolist())
    with open(os.path.join(HERE, "dip_64x64_degrees.txt"), "w") as fh:
        for j in range(M):
            fh.write(" ".join(str(v) for v in deg[j]) + "\n")


if __name__ == "__main__":
    main()
