"""Seeded test inputs shared by the CPU and GPU tests."""
import numpy as np

from paper_2606_12162_amd import workloads as W


def rough_case(nx, ny, bc, seed):
    rng = np.random.default_rng(seed)
    grid = W.Grid(nx, ny, 0.0, 0.0, 0.1, 0.13, bc)
    X, Y = W.cell_centres(grid)
    b = W.fp32_representable(-1.0 + 1.3 * X / X.max() + 0.1 * rng.standard_normal((ny, nx)))
    q = np.zeros((7, ny, nx))
    q[0] = np.maximum(0.1 * np.exp(-((X - 2) ** 2 + (Y - 3) ** 2)) - b, 0.0)
    q[1] = q[0] * 0.2 * rng.standard_normal((ny, nx))
    q[2] = q[0] * 0.2 * rng.standard_normal((ny, nx))
    q[3] = q[0] * 0.01 * rng.standard_normal((ny, nx))
    q[4] = q[0] * 0.01 * rng.standard_normal((ny, nx))
    q[5] = q[0] * q[0] * 0.05 * rng.standard_normal((ny, nx))
    q[6] = q[0] * q[0] * 0.05 * rng.standard_normal((ny, nx))
    P = W.Params(alpha=3.0, h_star=0.2, kappa=0.8)
    gx = np.array([[1.0, 1.0], [3.3, 2.1], [5.0, 4.0]])
    return W.Workload("rough_%dx%d_bc%s" % (nx, ny, "".join(map(str, bc))), P, grid, b, q, gx,
                      20, 0.004, 0.1)
