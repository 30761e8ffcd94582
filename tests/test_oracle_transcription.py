"""Second, independent transcription of one step (pure Python loops over
Sec. II, Eqs. (1), (2), (5)), compared with the C oracle on tiny lattices.

This checks the C code against the written steps; it is not a pin of the
readings (those are in test_oracle_physics.py / test_oracle_invariants.py).
The expected values here come from this file's own loops only.
"""
import math

import numpy as np
import pytest

import oracle
from paper_0906_3611_amd import inputs

C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
PCLASS = {1: 4 / 63, 2: 4 / 135, 4: 1 / 180, 5: 2 / 945, 8: 1 / 15120}
WCLASS = {1: 1 / 9, 2: 1 / 36}


def py_step(p, f):
    nx, ny = p.nx, p.ny
    rho = [[[sum(f[s][i][y][x] for i in range(9)) for x in range(nx)] for y in range(ny)] for s in range(2)]
    psi = [[[p.rho0 * (1 - math.exp(-rho[s][y][x] / p.rho0)) for x in range(nx)] for y in range(ny)]
           for s in range(2)]

    def row(y):
        if not p.walls:
            return y % ny
        return -1 - y if y < 0 else (2 * ny - 1 - y if y >= ny else y)

    out = [[[[0.0] * nx for _ in range(ny)] for _ in range(9)] for _ in range(2)]
    for y in range(ny):
        for x in range(nx):
            F = []
            for s in range(2):
                o = 1 - s
                fx = fy = 0.0
                for dy in range(-2, 3):
                    for dx in range(-2, 3):
                        c2 = dx * dx + dy * dy
                        if c2 == 0:
                            continue
                        yy, xx = row(y + dy), (x + dx) % nx
                        k = p.Ga[s] * WCLASS.get(c2, 0) + p.Gr[s] * PCLASS[c2]
                        kx = p.Gab / p.rho0 ** 2 * WCLASS.get(c2, 0)
                        val = -k * psi[s][y][x] * psi[s][yy][xx] - kx * rho[s][y][x] * rho[o][yy][xx]
                        fx += val * dx
                        fy += val * dy
                F.append((fx, fy))
            num = [0.0, 0.0]
            den = 0.0
            for s in range(2):
                jx = sum(f[s][i][y][x] * C[i][0] for i in range(9))
                jy = sum(f[s][i][y][x] * C[i][1] for i in range(9))
                num[0] += jx / p.tau[s]
                num[1] += jy / p.tau[s]
                den += rho[s][y][x] / p.tau[s]
            for s in range(2):
                r = rho[s][y][x]
                vx = num[0] / den + p.tau[s] * F[s][0] / r
                vy = num[1] / den + p.tau[s] * F[s][1] / r
                for i in range(9):
                    cu = 3 * (C[i][0] * vx + C[i][1] * vy)
                    feq = W[i] * r * (1 + cu + 0.5 * cu * cu - 1.5 * (vx * vx + vy * vy))
                    post = f[s][i][y][x] - (f[s][i][y][x] - feq) / p.tau[s]
                    yd = y + C[i][1]
                    if p.walls and not (0 <= yd < ny):
                        uw = p.u_wall if yd >= ny else -p.u_wall
                        j = C.index((-C[i][0], -C[i][1]))
                        out[s][j][y][x] = post - 6 * W[i] * r * C[i][0] * uw
                    else:
                        out[s][i][yd % ny][(x + C[i][0]) % nx] = post
    return np.array(out)


@pytest.mark.parametrize("walls", [False, True])
def test_oracle_matches_independent_transcription(walls):
    p = oracle.Params(nx=6, ny=7, tau=(0.9, 1.3), rho0=0.83, Ga=(-9.0, -8.0), Gr=(8.1, 7.1),
                      Gab=0.405, walls=walls, u_wall=0.03 if walls else 0.0)
    ra, rb = inputs.noise_fields(6, 7, 21, 0.6, 0.45, 0.1)
    f = oracle.init_equilibrium(p, ra, rb)
    f = oracle.step(p, f)  # start from a non-equilibrium state
    a = oracle.step(p, f)
    b = py_step(p, f.tolist())
    assert np.abs(a - b).max() < 1e-14
