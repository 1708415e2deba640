"""Per-node oracle of one time step, in pull form (test infrastructure only).

A second implementation of the step of scheme.py that visits nodes one at a
time with explicit index arithmetic instead of whole-array rolls and padding:

  * streaming is a pull, f_i(x) = f_post_i(x - c_i) (Eq. pushLB read
    backwards), with half-way bounce-back f_i(x) = f_post_opp(i)(x) when
    x - c_i lies behind a wall (reading R11 of scheme.py);
  * ghost nodes are resolved by mapping every coordinate through the
    periodic wrap or the half-way mirror, and the ghost velocity and normal
    get their reflection signs node by node.

The local physics (density, forces, equilibria, regularisation, source) is the
one of scheme.py, evaluated on single nodes.  FinePointOracle does the same for
the finer phase-field grid (scheme.py F1-F5): the fine FTCS update node by node,
the coarse u interpolated per fine node, and the restriction per coarse cell.  Used on tiny grids to check the
streaming and boundary indexing of scheme.py, and on sampled nodes of full-size
problems where the whole-array oracle does not fit in memory.
"""
from __future__ import annotations

import numpy as np

from . import scheme
from .lattice import C, CS2, OPP, Q as NQ, W

PERIODIC = scheme.PERIODIC


class PointOracle:
    """Evaluates one step at chosen nodes from a full state held on the host."""

    def __init__(self, st, prob):
        self.st = st
        self.prob = prob
        self.n = (prob.nx, prob.ny, prob.nz)
        self._cache = {}

    # -- coordinates ---------------------------------------------------------
    def _map(self, ax, i):
        """Map coordinate i on axis ax into the domain.  Returns (index, mirrored)."""
        n = self.n[ax]
        if self.prob.bc[ax] == PERIODIC:
            return i % n, False
        if i < 0:
            return -1 - i, True
        if i >= n:
            return 2 * n - 1 - i, True
        return i, False

    def _inside(self, ax, i):
        return self.prob.bc[ax] == PERIODIC or 0 <= i < self.n[ax]

    def phi_at(self, x, y, z):
        xs = self._map(0, x)[0]
        ys = self._map(1, y)[0]
        zs = self._map(2, z)[0]
        return self.st.phi[zs, ys, xs]

    def J_at(self, x, y, z):
        """J at a node that may be a ghost: minus the mirrored value per crossed wall (R11)."""
        xs, mx = self._map(0, x)
        ys, my = self._map(1, y)
        zs, mz = self._map(2, z)
        return self.st.J[:, zs, ys, xs] * (-1.0) ** (mx + my + mz)

    # -- node quantities at an in-domain node ---------------------------------
    def node(self, x, y, z):
        key = (x, y, z)
        if key in self._cache:
            return self._cache[key]
        prob, st = self.prob, self.st
        phi = st.phi[z, y, x]
        gphi = np.zeros(3)
        lap = 0.0
        rho_c = scheme.density(phi, prob)
        for i in range(NQ):
            cx, cy, cz = (int(v) for v in C[i])
            pn = self.phi_at(x + cx, y + cy, z + cz)
            gphi += (W[i] / CS2) * pn * C[i]
            lap += (2.0 * W[i] / CS2) * (pn - phi)
        grho = scheme.density_gradient(gphi, prob)
        P = st.P[z, y, x]
        J = st.J[:, z, y, x].copy()
        om = scheme.relaxation(scheme.viscosity(phi, prob))
        if prob.gradient_closure:
            # a2 from the isotropic gradient of J, neighbours by index (G1-G3)
            gJ = np.zeros((3, 3))
            for i in range(NQ):
                cx, cy, cz = (int(v) for v in C[i])
                gJ += (W[i] / CS2) * np.outer(self.J_at(x + cx, y + cy, z + cz), C[i])
            A = -(CS2 / om) * (gJ + gJ.T)
            F = scheme.total_force(np.float64(phi), gphi, np.float64(lap), grho,
                                   np.float64(P), A, prob)
            fpost, u, A, a = scheme.collide_closed(np.float64(P), J, A, F, rho_c, om)
        else:
            Qt = st.Q[:, :, z, y, x].copy()
            F = scheme.total_force(np.float64(phi), gphi, np.float64(lap), grho,
                                   np.float64(P), Qt, prob)
            fpost, u, A, a = scheme.collide(np.float64(P), J, Qt, F, rho_c, om)
        mag = np.sqrt(np.sum(gphi ** 2))
        res = dict(phi=phi, grad_phi=gphi, lap=lap, u=u, fpost=fpost,
                   n=gphi / (mag + scheme.EPS_NORMAL))
        self._cache[key] = res
        return res

    def flux_parts(self, x, y, z):
        """(phi, u, n) at a node that may be a ghost, with reflection signs."""
        xs, mx = self._map(0, x)
        ys, my = self._map(1, y)
        zs, mz = self._map(2, z)
        q = self.node(xs, ys, zs)
        crossed = (mx, my, mz)
        u = q["u"] * (-1.0) ** sum(crossed)
        n = q["n"] * np.array([-1.0 if m else 1.0 for m in crossed])
        return q["phi"], u, n

    # -- fourth-order phase-field stencils (scheme.py H1, H3) ------------------
    def grad4_at(self, x, y, z):
        """(4 D_1 - D_2)/3 of phi at in-domain node (x, y, z): D_1 over the
        neighbours x + c_i, D_2 over x + 2 c_i with half the weight."""
        key = ("g4", x, y, z)
        if key in self._cache:
            return self._cache[key]
        g1 = np.zeros(3)
        g2 = np.zeros(3)
        for i in range(NQ):
            cx, cy, cz = (int(v) for v in C[i])
            g1 += (W[i] / CS2) * self.phi_at(x + cx, y + cy, z + cz) * C[i]
            g2 += (W[i] / (2.0 * CS2)) * self.phi_at(x + 2 * cx, y + 2 * cy, z + 2 * cz) * C[i]
        g = (4.0 * g1 - g2) / 3.0
        self._cache[key] = g
        return g

    def flux_parts4(self, x, y, z):
        """(phi, u, n4) at a node that may be a ghost: the mirrored node's
        values, u negated per crossed wall, n4's crossed components negated."""
        xs, mx = self._map(0, x)
        ys, my = self._map(1, y)
        zs, mz = self._map(2, z)
        q = self.node(xs, ys, zs)
        g = self.grad4_at(xs, ys, zs)
        n = g / (np.sqrt(np.sum(g ** 2)) + scheme.EPS_NORMAL)
        crossed = (mx, my, mz)
        u = q["u"] * (-1.0) ** sum(crossed)
        n = n * np.array([-1.0 if m else 1.0 for m in crossed])
        return q["phi"], u, n

    def phase_high_order_at(self, x, y, z):
        """phi' at (x, y, z) with the fourth-order stencils (scheme.py H1)."""
        prob = self.prob
        own = self.node(x, y, z)
        kac = 4.0 * prob.mobility / prob.width
        adv = [0.0, 0.0]
        sharp = [0.0, 0.0]
        lap = [0.0, 0.0]
        for i in range(NQ):
            cx, cy, cz = (int(v) for v in C[i])
            for s in (1, 2):
                ph, u, n = self.flux_parts4(x + s * cx, y + s * cy, z + s * cz)
                wt = W[i] / (s * CS2)
                adv[s - 1] += wt * ph * float(np.dot(u, C[i]))
                sharp[s - 1] += wt * ph * (1.0 - ph) * float(np.dot(n, C[i]))
                lap[s - 1] += (2.0 * W[i] / (s * s * CS2)) * (
                    self.phi_at(x + s * cx, y + s * cy, z + s * cz) - own["phi"])
        four = lambda v: (4.0 * v[0] - v[1]) / 3.0
        if prob.literal_advection:
            a = float(np.dot(own["u"], self.grad4_at(x, y, z)))
        else:
            a = four(adv)
        return own["phi"] - a + prob.mobility * four(lap) - kac * four(sharp)

    # -- one step at one node -------------------------------------------------
    def step_at(self, x, y, z):
        """Returns (phi', P', J'(3), Q'(3x3)) at in-domain node (x, y, z)."""
        prob = self.prob
        own = self.node(x, y, z)
        f = np.empty(NQ)
        for i in range(NQ):
            cx, cy, cz = (int(v) for v in C[i])
            src = (x - cx, y - cy, z - cz)
            if all(self._inside(ax, src[ax]) for ax in range(3)):
                xs = self._map(0, src[0])[0]
                ys = self._map(1, src[1])[0]
                zs = self._map(2, src[2])[0]
                f[i] = self.node(xs, ys, zs)["fpost"][i]
            else:
                f[i] = own["fpost"][OPP[i]]
        P = f.sum()
        J = C.T.astype(np.float64) @ f
        Pi = np.einsum("i,ia,ib->ab", f, C.astype(np.float64), C.astype(np.float64))
        Qn = Pi - CS2 * P * np.eye(3) - np.outer(J, J)
        if prob.gradient_closure:
            Qn = np.zeros((3, 3))  # not part of the state (G4)

        kac = 4.0 * prob.mobility / prob.width
        div_adv = 0.0
        div_sharp = 0.0
        for i in range(NQ):
            cx, cy, cz = (int(v) for v in C[i])
            ph, u, n = self.flux_parts(x + cx, y + cy, z + cz)
            div_adv += (W[i] / CS2) * ph * float(np.dot(u, C[i]))
            div_sharp += (W[i] / CS2) * ph * (1.0 - ph) * float(np.dot(n, C[i]))
        if prob.literal_advection:
            adv = float(np.dot(own["u"], own["grad_phi"]))
        else:
            adv = div_adv
        phi_new = own["phi"] - adv + prob.mobility * own["lap"] - kac * div_sharp
        if getattr(prob, "high_order_ac", False):
            phi_new = self.phase_high_order_at(x, y, z)
        return phi_new, P, J, Qn


# -- finer phase-field grid (scheme.py F1-F5), node by node --------------------
def _map_index(periodic, n, i):
    """Coordinate i of an axis of n nodes mapped into the domain: wrapped if
    periodic, else mirrored half-way (-1 -> 0).  Returns (index, mirrored)."""
    if periodic:
        return i % n, False
    if i < 0:
        return -1 - i, True
    if i >= n:
        return 2 * n - 1 - i, True
    return i, False


def prolong_at(g_at, prob, X, Y, Z, odd=False):
    """Trilinear interpolation (F3) of a coarse field at in-domain fine node
    (X, Y, Z) (F1: fine node I of an axis at I/2 - 1/4): per axis the coarse
    node I // 2 with weight 3/4 and its neighbour on the fine node's side
    (I even: below, I odd: above) with weight 1/4.  g_at(x, y, z) reads an
    in-domain coarse node; a coarse node beyond a wall takes the mirrored
    node's value, negated per crossed wall when odd."""
    n = (prob.nx, prob.ny, prob.nz)
    taps = []
    for ax, I in enumerate((X, Y, Z)):
        c = I // 2
        taps.append(((c, 0.75), (c - 1 if I % 2 == 0 else c + 1, 0.25)))
    total = 0.0
    for cx, wx in taps[0]:
        for cy, wy in taps[1]:
            for cz, wz in taps[2]:
                idx, crossed = [], 0
                for ax, c in enumerate((cx, cy, cz)):
                    i, m = _map_index(prob.bc[ax] == PERIODIC, n[ax], c)
                    idx.append(i)
                    crossed += m
                v = g_at(*idx)
                if odd and crossed % 2:
                    v = -v
                total = total + (wx * wy * wz) * v
    return total


class FinePointOracle:
    """One step of scheme.step_fine evaluated at chosen coarse nodes.

    st is the coarse state of level n, whose phi is the restriction of the
    fine field (F2); phif_at(X, Y, Z) reads the fine phi at an in-domain fine
    node.  The coarse part of the step (collision, streaming, moments) is
    PointOracle's; the new coarse phi is the mean of the 8 fine nodes of the
    cell after the fine FTCS update (F4), whose fluxes use the interpolated
    coarse u of level n (F3) and, beyond a wall, the mirrored fine node with u
    negated per crossed wall and the gradient taken on the mirrored field
    (F5)."""

    def __init__(self, st, phif_at, prob):
        self.coarse = PointOracle(st, prob)
        self.phif_at = phif_at
        self.prob = prob
        self.nf = (2 * prob.nx, 2 * prob.ny, 2 * prob.nz)
        self._cache = {}

    def _map(self, ax, i):
        return _map_index(self.prob.bc[ax] == PERIODIC, self.nf[ax], i)

    def phi_at(self, X, Y, Z):
        """Fine phi at a fine node that may be a ghost (mirrored value)."""
        return self.phif_at(self._map(0, X)[0], self._map(1, Y)[0], self._map(2, Z)[0])

    def u_at(self, X, Y, Z):
        """Interpolated coarse u at an in-domain fine node (F3)."""
        key = ("u", X, Y, Z)
        if key not in self._cache:
            self._cache[key] = prolong_at(lambda x, y, z: self.coarse.node(x, y, z)["u"], self.prob,
                                          X, Y, Z, odd=True)
        return self._cache[key]

    def grad_at(self, X, Y, Z):
        """Isotropic gradient of the fine phi at spacing h (Sec. II.C stencil
        divided by h) at a fine node that may be a ghost."""
        key = ("g", X, Y, Z)
        if key not in self._cache:
            g = np.zeros(3)
            for i in range(NQ):
                cx, cy, cz = (int(v) for v in C[i])
                g += (W[i] / CS2) * self.phi_at(X + cx, Y + cy, Z + cz) * C[i]
            self._cache[key] = g / scheme.FINE_H
        return self._cache[key]

    def flux_parts(self, X, Y, Z):
        """(phi, u, n) at a fine node that may be a ghost (F5)."""
        idx, crossed = [], 0
        for ax, I in enumerate((X, Y, Z)):
            i, m = self._map(ax, I)
            idx.append(i)
            crossed += m
        u = self.u_at(*idx) * (-1.0) ** crossed
        g = self.grad_at(X, Y, Z)
        n = g / (np.sqrt(np.sum(g ** 2)) + scheme.EPS_NORMAL)
        return self.phif_at(*idx), u, n

    def phase_at(self, X, Y, Z):
        """phi_f' at an in-domain fine node: the FTCS update of Sec. II.D with
        the divergence divided by h and the Laplacian by h^2 (F4)."""
        prob, h = self.prob, scheme.FINE_H
        kac = 4.0 * prob.mobility / prob.width
        ph0 = self.phif_at(X, Y, Z)
        adv = sharp = lap = 0.0
        for i in range(NQ):
            cx, cy, cz = (int(v) for v in C[i])
            ph, u, n = self.flux_parts(X + cx, Y + cy, Z + cz)
            adv += (W[i] / CS2) * ph * float(np.dot(u, C[i]))
            sharp += (W[i] / CS2) * ph * (1.0 - ph) * float(np.dot(n, C[i]))
            lap += (2.0 * W[i] / CS2) * (ph - ph0)
        return ph0 - adv / h + prob.mobility * lap / (h * h) - kac * sharp / h

    def step_at(self, x, y, z):
        """(phi', P', J'(3), Q'(3x3)) at in-domain coarse node (x, y, z);
        phi' is the restriction of the 8 updated fine nodes (F2)."""
        _, P, J, Qn = self.coarse.step_at(x, y, z)
        kids = [self.phase_at(2 * x + dx, 2 * y + dy, 2 * z + dz)
                for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        return float(np.mean(kids)), P, J, Qn


def step_points_fine(st, phif_at, prob, points):
    """step_points for the finer phase grid (FinePointOracle)."""
    po = FinePointOracle(st, phif_at, prob)
    out = dict(phi=[], P=[], J=[], Q=[])
    for (x, y, z) in points:
        phi, P, J, Qn = po.step_at(int(x), int(y), int(z))
        out["phi"].append(phi)
        out["P"].append(P)
        out["J"].append(J)
        out["Q"].append(Qn)
    return {k: np.array(v) for k, v in out.items()}


def step_points(st, prob, points):
    """One step evaluated at a list of (x, y, z) nodes.  Returns dict of arrays."""
    po = PointOracle(st, prob)
    out = dict(phi=[], P=[], J=[], Q=[])
    for (x, y, z) in points:
        phi, P, J, Qn = po.step_at(int(x), int(y), int(z))
        out["phi"].append(phi)
        out["P"].append(P)
        out["J"].append(J)
        out["Q"].append(Qn)
    return {k: np.array(v) for k, v in out.items()}


def step_full(st, prob):
    """Whole-grid step by visiting every node (tiny grids only)."""
    nz, ny, nx = st.phi.shape
    po = PointOracle(st, prob)
    phi = np.empty_like(st.phi)
    P = np.empty_like(st.P)
    J = np.empty_like(st.J)
    Qt = np.empty_like(st.Q)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                a, b, c, d = po.step_at(x, y, z)
                phi[z, y, x] = a
                P[z, y, x] = b
                J[:, z, y, x] = c
                Qt[:, :, z, y, x] = d
    return scheme.State(phi, P, J, Qt)
