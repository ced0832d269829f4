"""Pins of the oracle's periodic-boundary error E (sec. 2.7, eq. relativeErrorPbc).

E is taken per cell on the periodic inflow summed over directions (per group),
E_c = |j^n - j^{n-1}| / (j^n + j^{n-1}) between the last two passes, reported as
its maximum over cells (totals[6]) and in L1 form (totals[7]).  On a periodic
cubic lattice with axis-aligned directions every transverse face is parallel to
the direction (it carries nothing), so each row of cells along the direction is
an independent chain closed on itself through one periodic face:

    phi_0 = a_0 (b + sigma),   phi_i = a_i phi_{i-1},   a_i = 1 / (1 + kappa_i h)

(cell balance (A + kappa V) phi = A phi_up + S with A = h^2, V = h^3, and
sigma = S / h^2 for the source in cell 0).  The inflow b of pass p is what
left the chain's last cell in pass p - 1, b^0 = 0, so with q = prod_i a_i

    b^p = sigma (q + q^2 + ... + q^p) = sigma q (1 - q^p) / (1 - q)

and the periodic inflow of cell 0 is h^2 b^p.  The cases below need each
ingredient of E: the sum over directions before the ratio (two chains of
different transmission meeting in one cell), the maximum against the L1 form
(two cells), and the pass indices (several pass counts)."""
import numpy as np
import pytest

import oracle
from synth.mesh import lattice_mesh

N = 8
H = 1.0 / N


def cid(i, j, k):
    return i + N * (j + N * k)


def b_closed(p, sigma, q):
    """Periodic inflow (per unit w) of the chain's first cell in pass p."""
    return sigma * q * (1.0 - q ** p) / (1.0 - q)


def run(kappa, emission, dirs, n_pbc):
    w = dict(meshes=[lattice_mesh(N, periodic=True)], dirs=np.asarray(dirs, np.float64), G=1,
             kappa=np.asarray(kappa, np.float64).reshape(-1, 1),
             emission=np.asarray(emission, np.float64).reshape(-1, 1), boundary="periodic",
             n_pbc=n_pbc, albedo=0.0, n_scat=1)
    t = oracle.forward(w)["totals"][0, 0]
    return t[6], t[7]


@pytest.mark.parametrize("n_pbc", [2, 3, 4, 6])
def test_single_chain_geometric_series(n_pbc):
    """One direction (+x), one source, uniform kappa: E = q^{P-2}(1-q)/(2 - q^{P-1} - q^{P-2})."""
    kap = 0.5
    C = N ** 3
    em = np.zeros(C)
    em[cid(0, 3, 5)] = 1.0
    emax, el1 = run(np.full(C, kap), em, [[1.0, 0.0, 0.0]], n_pbc)
    q = (1.0 / (1.0 + kap * H)) ** N
    P = n_pbc
    expect = q ** (P - 2) * (1 - q) / (2 - q ** (P - 1) - q ** (P - 2))
    # and the same from the series itself
    sigma = 1.0 / H ** 2
    jn, jo = H * H * b_closed(P - 1, sigma, q), H * H * b_closed(P - 2, sigma, q)
    assert abs(expect - (jn - jo) / (jn + jo)) <= 1e-11 * expect
    assert abs(emax - expect) <= 1e-12 * expect
    assert abs(el1 - expect) <= 1e-12 * expect
    if P == 2:
        assert abs(emax - 1.0) <= 1e-15


def test_directions_summed_before_the_ratio():
    """Two directions (+x, +y) whose chains through the source cell transmit
    differently (kappa_x along the row, kappa_y along the column): the source
    cell's inflow is the sum of both chains' outflow, and E is the ratio of the
    summed change to the summed inflow, not a per-direction ratio."""
    C = N ** 3
    k0, kx, ky, kr = 1.5, 0.5, 6.0, 2.0
    kap = np.full(C, kr)
    src = cid(0, 0, 2)
    for i in range(1, N):
        kap[cid(i, 0, 2)] = kx
    for j in range(1, N):
        kap[cid(0, j, 2)] = ky
    kap[src] = k0
    em = np.zeros(C)
    em[src] = 2.0
    D = 2
    sigma = (2.0 / D) / H ** 2
    a0, ax, ay = 1 / (1 + k0 * H), 1 / (1 + kx * H), 1 / (1 + ky * H)
    qx, qy = a0 * ax ** (N - 1), a0 * ay ** (N - 1)
    for P in (3, 5):
        emax, el1 = run(kap, em, [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]], P)
        jn = H * H * (b_closed(P - 1, sigma, qx) + b_closed(P - 1, sigma, qy))
        jo = H * H * (b_closed(P - 2, sigma, qx) + b_closed(P - 2, sigma, qy))
        expect = (jn - jo) / (jn + jo)
        assert abs(emax - expect) <= 1e-12 * expect
        assert abs(el1 - expect) <= 1e-12 * expect
        # a per-direction reading would give something else
        ex = [(b_closed(P - 1, 1, q) - b_closed(P - 2, 1, q)) /
              (b_closed(P - 1, 1, q) + b_closed(P - 2, 1, q)) for q in (qx, qy)]
        for e in ex + [max(ex), sum(ex) / 2]:
            assert abs(e - expect) > 1e-3 * expect


def test_maximum_and_l1_forms():
    """One direction, two sources in different rows of different opacity: the
    maximum picks the slower-converging cell, the L1 form divides the summed
    changes by the summed inflows."""
    C = N ** 3
    kap = np.full(C, 1.0)
    r1, r2 = (1, 1), (5, 6)
    k1, k2 = 0.4, 4.0
    L1, L2 = 1.0, 3.0
    for i in range(N):
        kap[cid(i, *r1)] = k1
        kap[cid(i, *r2)] = k2
    em = np.zeros(C)
    em[cid(0, *r1)] = L1
    em[cid(0, *r2)] = L2
    q1, q2 = (1 / (1 + k1 * H)) ** N, (1 / (1 + k2 * H)) ** N
    for P in (2, 3, 4):
        emax, el1 = run(kap, em, [[1.0, 0.0, 0.0]], P)
        d, s, e = [], [], []
        for q, L in ((q1, L1), (q2, L2)):
            sg = L / H ** 2
            jn, jo = H * H * b_closed(P - 1, sg, q), H * H * b_closed(P - 2, sg, q)
            d.append(jn - jo)
            s.append(jn + jo)
            e.append((jn - jo) / (jn + jo))
        assert abs(emax - max(e)) <= 1e-12 * max(e)
        l1 = sum(d) / sum(s)
        assert abs(el1 - l1) <= 1e-12 * l1
        if P > 2:
            assert abs(e[0] - e[1]) > 1e-2 and abs(l1 - max(e)) > 1e-3


def test_single_pass_reports_zero():
    C = N ** 3
    em = np.zeros(C)
    em[cid(0, 0, 0)] = 1.0
    emax, el1 = run(np.full(C, 1.0), em, [[1.0, 0.0, 0.0]], 1)
    assert emax == 0.0 and el1 == 0.0
