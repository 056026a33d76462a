"""Writes grid2d_32_nev50.txt: the 50 smallest eigenvalues of the 32 x 32
Dirichlet 5-point Laplacian A = I (x) T + T (x) I, T = tridiag(-1, 2, -1),
from the closed form lambda_{j,k} = 4 sin^2(j pi / 66) + 4 sin^2(k pi / 66)
(separable eigenvectors sin(j pi x / 33) sin(k pi y / 33)), with the
multiplicity of each value.  Run from the repository root:
    python tests/golden/make_grid2d_32.py
"""
import os

import numpy as np

n = 32
j = np.arange(1, n + 1)
s = 4.0 * np.sin(j * np.pi / (2 * (n + 1))) ** 2
lam = np.sort((s[:, None] + s[None, :]).ravel())
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid2d_32_nev50.txt")
with open(out, "w") as f:
    f.write("# 50 smallest eigenvalues of the 32x32 Dirichlet grid Laplacian (closed form),\n")
    f.write("# written by tests/golden/make_grid2d_32.py; lambda_51 follows as a gap check\n")
    for v in lam[:51]:
        f.write("%.17e\n" % v)
