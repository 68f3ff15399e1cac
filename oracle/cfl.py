"""Explicit (leap-frog) stability limit of the Kuhn cube meshes, FP64 (test infrastructure).

dt_CFL = 2 / sqrt(lambda_max([*eps]^-1 S)) on the interior edges. The lattice is
self-similar, so n * dt_CFL(n) converges as n grows; the 64^3 limit is taken as the
16^3 value scaled by 16/64 (the 8^3 -> 16^3 change of n * dt_CFL is 0.8%).

    python -m oracle.cfl      prints dt_CFL for n = 8, 16 and the 64^3 estimate
"""
import numpy as np

import qh_inputs as qi

from .complex_ import Complex
from .field import dt_cfl
from .whitney import Operators


def kuhn_dt_cfl(n: int) -> float:
    m = qi.BoxMesh(n)
    cx = Complex(m.xyz, m.tets)
    return dt_cfl(Operators(cx, qi.EPS0, qi.MU0), cx, tol=1e-6)


if __name__ == "__main__":
    d8, d16 = kuhn_dt_cfl(8), kuhn_dt_cfl(16)
    print(f"n=8  dt_cfl={d8:.6e}  n*dt={8 * d8:.6e}")
    print(f"n=16 dt_cfl={d16:.6e}  n*dt={16 * d16:.6e}")
    print(f"n=64 estimate dt_cfl={16 * d16 / 64:.6e}; 10x = {10 * 16 * d16 / 64:.6e}")
