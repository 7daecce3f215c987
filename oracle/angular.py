"""Angular discretisation (oracle; test infrastructure only).

Follows Section 2.1 (patches obtained by recursively splitting the eight
octant triangles into four daughters through great-circle edge midpoints),
Section 2.2 (the Lin basis: nodal functions that are the Lagrange functions
of the flat triangle spanned by the patch vertices projected onto the
octahedron face; and the Const basis, one constant per patch), Section 4.1 (nested meshes T_l, two-irregularity, Galerkin
prolongation with R = P^T), Section 5.2 (the harmonic expansion of the
scatter source and the X integrals of eq. X) and Section 5.5 (the z-band
anisotropic refinement rule with its element counts).

Readings where the paper is silent (each also listed in the design notes):
  * projection onto the octahedron face is the central (gnomonic) one,
    x -> x / (s . x) for octant sign vector s;
  * the transport terms (M, A^xi and the source/detector integrals of psi)
    use a 3-point rule per patch: points at barycentric (2/3, 1/6, 1/6) of
    the flat triangle mapped to the sphere, weights that integrate the
    three Lin functions exactly.  Three points for three functions make the
    rule collocated, so each (cell, patch) block decouples into three
    ordinates after a fixed 3x3 change of basis;
  * the Const basis' transport terms (M_q = |q|, A^xi_q = int_q Omega_xi,
    int psi = |q|) are integrated with the accurate rule below;
  * the X integrals of eq. X are integrals: they are evaluated with a
    high-order (collapsed Gauss) rule to round-off.  Evaluating them with
    the 3-point rule aliases high Legendre orders on coarse meshes (the
    discrete scatter operator then amplifies, spectral radius up to 8 on
    T_0 at order 16) and the coarse problems stop being transport problems;
  * refinement rules are evaluated at the patch vertices;
  * patch order is octant-major (octant id = [s_x<0] + 2[s_y<0] + 4[s_z<0])
    then depth-first over the children in split order.
"""
import math
import numpy as np


# ---------------------------------------------------------------- patches

def octant_signs(octant):
    """Sign vector s of octant id o = [s_x<0] + 2[s_y<0] + 4[s_z<0]."""
    return np.array([-1.0 if octant & 1 else 1.0,
                     -1.0 if octant & 2 else 1.0,
                     -1.0 if octant & 4 else 1.0])


def great_circle_midpoint(a, b):
    m = a + b
    return m / np.linalg.norm(m)


class Patch:
    """A spherical triangle D_p with its three vertices (rows of ``verts``),
    refinement level l_p, octant, parent and (after a split) four children."""

    def __init__(self, verts, level, octant, parent=None):
        self.verts = np.array(verts, dtype=np.float64)
        self.level = level
        self.octant = octant
        self.parent = parent
        self.children = None

    def split(self):
        """Halve the edges with great circles: four daughters (Section 2.1)."""
        a, b, c = self.verts
        mab = great_circle_midpoint(a, b)
        mbc = great_circle_midpoint(b, c)
        mca = great_circle_midpoint(c, a)
        kids = [(a, mab, mca), (mab, b, mbc), (mca, mbc, c), (mab, mbc, mca)]
        self.children = [Patch(v, self.level + 1, self.octant, self) for v in kids]
        return self.children

    def ancestor_at(self, level):
        p = self
        while p.level > level:
            p = p.parent
        return p


def spherical_area(verts):
    """Exact area of a spherical triangle (Van Oosterom & Strackee)."""
    a, b, c = verts
    num = abs(np.dot(a, np.cross(b, c)))
    den = 1.0 + np.dot(a, b) + np.dot(b, c) + np.dot(c, a)
    return 2.0 * math.atan2(num, den)


# ------------------------------------------------------------ refinement

def uniform_rule(level):
    return lambda verts: level


def band_z_rule(lmax):
    """Section 5.5: level lmax where Omega_z > 0.97, lmax-1 above 0.9, lmax-2
    above 0.8, lmax-3 above 0.6, lmax-4 elsewhere (clamped at 0), each test
    applied to the largest vertex Omega_z of the element."""
    def rule(verts):
        z = verts[:, 2].max()
        if z > 0.97:
            lev = lmax
        elif z > 0.9:
            lev = lmax - 1
        elif z > 0.8:
            lev = lmax - 2
        elif z > 0.6:
            lev = lmax - 3
        else:
            lev = lmax - 4
        return max(lev, 0)
    return rule


def cone_rule(axis, half_angle_deg, base_level, extra_levels):
    """Base level everywhere plus ``extra_levels`` where any vertex lies
    strictly inside the cone of the given half angle around ``axis``."""
    ax = np.asarray(axis, dtype=np.float64)
    ax = ax / np.linalg.norm(ax)
    cth = math.cos(math.radians(half_angle_deg))

    def rule(verts):
        inside = (verts @ ax > cth).any()
        return base_level + (extra_levels if inside else 0)
    return rule


def edge_neighbours(leaves, tol=1e-12):
    """Pairs (i, j) of leaves sharing a boundary segment of positive length.
    On a hierarchical mesh a shared segment is a whole edge of the finer of
    the two patches, so it suffices to test whether the midpoint of one
    patch's edge lies strictly inside an edge of the other (the minor arc
    u-v contains m when the angles u-m and m-v add up to u-v)."""
    U, V, owner = [], [], []
    for idx, p in enumerate(leaves):
        for e in range(3):
            U.append(p.verts[e])
            V.append(p.verts[(e + 1) % 3])
            owner.append(idx)
    U, V, owner = np.array(U), np.array(V), np.array(owner)
    M = U + V
    M /= np.linalg.norm(M, axis=1)[:, None]
    ang = lambda a, b: np.arccos(np.clip(a @ b.T, -1.0, 1.0))
    a_uv = np.arccos(np.clip(np.sum(U * V, axis=1), -1.0, 1.0))[None, :]
    a_um = ang(M, U)            # [i, j]: midpoint of edge i vs start of edge j
    a_mv = ang(M, V)
    hit = (np.abs(a_um + a_mv - a_uv) < tol) & (a_um > tol) & (a_mv > tol)
    hit &= owner[:, None] != owner[None, :]
    i, j = np.nonzero(hit)
    pairs = {(min(a, b), max(a, b)) for a, b in zip(owner[i], owner[j])}
    return sorted(pairs)


class AngularMesh:
    """The patch tree: eight level-0 octant triangles refined by a rule."""

    def __init__(self, rule, closure=False):
        self.roots = []
        for o in range(8):
            s = octant_signs(o)
            self.roots.append(Patch(np.diag(s), 0, o))
        self._apply_rule(rule)
        if closure:
            # Section 4.1: neighbouring elements differ by two levels at most.
            while True:
                leaves = self.leaves()
                todo = set()
                for i, j in edge_neighbours(leaves):
                    li, lj = leaves[i].level, leaves[j].level
                    if li - lj > 2:
                        todo.add(j)
                    elif lj - li > 2:
                        todo.add(i)
                if not todo:
                    break
                for k in todo:
                    leaves[k].split()
                self._apply_rule(rule)

    def _apply_rule(self, rule):
        stack = list(self.leaves())
        while stack:
            p = stack.pop()
            if p.level < rule(p.verts):
                stack.extend(p.split())

    @classmethod
    def uniform(cls, level):
        return cls(uniform_rule(level))

    @classmethod
    def band_z(cls, lmax):
        return cls(band_z_rule(lmax))

    @classmethod
    def cone(cls, axis, half_angle_deg, base_level, extra_levels, closure=True):
        return cls(cone_rule(axis, half_angle_deg, base_level, extra_levels), closure=closure)

    def _dfs(self, p, cut):
        if p.children is None or p.level == cut:
            yield p
        else:
            for c in p.children:
                yield from self._dfs(c, cut)

    def leaves(self, cut=10 ** 9):
        """Leaves of the tree truncated at level ``cut``, octant-major then
        depth-first in split order."""
        out = []
        for r in self.roots:
            out.extend(self._dfs(r, cut))
        return out

    @property
    def max_level(self):
        return max(p.level for p in self.leaves())

    def levels(self):
        """Nested meshes T_0 ... T_L (Section 4.1): T_l holds the leaves of
        the tree cut at level l."""
        return [self.leaves(cut=l) for l in range(self.max_level + 1)]


# -------------------------------------------------------------- Lin basis

def gnomonic(points, s):
    """Central projection onto the octahedron face plane s . x = 1."""
    points = np.atleast_2d(points)
    return points / (points @ s)[:, None]


def lin_basis(patch, omegas):
    """psi_{[p]d}(Omega) for the Lin set (Section 2.2): barycentric
    coordinates of the projected direction in the flat triangle spanned by
    the projected patch vertices.  Returns shape (npoints, 3)."""
    s = octant_signs(patch.octant)
    flat = gnomonic(patch.verts, s)              # rows: projected vertices
    x = gnomonic(np.asarray(omegas, float), s)
    # columns of flat.T are the flat vertices; points on the plane s.x = 1
    # have barycentric coordinates summing to one automatically.
    return np.linalg.solve(flat.T, x.T).T


def const_basis(patch, omegas):
    """psi_q = 1 on the patch: the Const set of Section 2.2 (one dof per
    patch).  Returns shape (npoints, 1)."""
    return np.ones((len(np.atleast_2d(omegas)), 1))


# angular bases: name -> (basis function, dofs per patch)
BASES = {"lin": (lin_basis, 3), "const": (const_basis, 1)}


def basis_dofs(basis):
    return BASES[basis][1]


# ------------------------------------------------------------ quadrature

def _flat_rule_on_patch(patch, bary, bary_w):
    """Map a rule given on the flat (projected) triangle to the sphere with
    the gnomonic Jacobian dOmega = dA / (sqrt(3) |x|^3) (the face plane
    s . x = 1 lies at distance 1/sqrt(3) from the origin).  ``bary_w`` are
    weights normalised to a unit-area triangle."""
    s = octant_signs(patch.octant)
    flat = gnomonic(patch.verts, s)
    x = bary @ flat
    r = np.linalg.norm(x, axis=1)
    area_flat = 0.5 * np.linalg.norm(np.cross(flat[1] - flat[0], flat[2] - flat[0]))
    w = area_flat * bary_w / (math.sqrt(3.0) * r ** 3)
    return x / r[:, None], w


def collapsed_gauss(n):
    """n x n Gauss-Legendre points on the unit square collapsed onto the
    reference triangle (Duffy map b1 = u, b2 = v (1 - u)); weights sum to 1."""
    t, wt = np.polynomial.legendre.leggauss(n)
    u, wu = (t + 1) / 2, wt / 2
    U, V = np.meshgrid(u, u, indexing='ij')
    WU, WV = np.meshgrid(wu, wu, indexing='ij')
    b1 = U.ravel()
    b2 = (V * (1 - U)).ravel()
    w = 2.0 * (WU * WV * (1 - U)).ravel()
    return np.stack([1 - b1 - b2, b1, b2], axis=1), w


def patch_angle(patch):
    """Largest angle between two vertices of the patch."""
    a, b, c = patch.verts
    return max(math.acos(min(1.0, float(np.dot(u, v)))) for u, v in ((a, b), (b, c), (c, a)))


def accurate_points(order, patch):
    """Gauss order per direction for integrands psi * Y_n, n <= order: the
    collapsed rule converges exponentially; this count keeps the integrals
    at round-off for the oscillation a degree-``order`` harmonic has across
    the patch."""
    th = patch_angle(patch)
    return int(min(96, max(16, math.ceil(10 + 8 * th + 1.5 * order * th))))


def quad_accurate(patch, order=0):
    """Reference integration rule on a patch, accurate for psi * Y_{n<=order}."""
    bary, w = collapsed_gauss(accurate_points(order, patch))
    return _flat_rule_on_patch(patch, bary, w)


QUAD3_BARY = np.array([[2 / 3, 1 / 6, 1 / 6],
                       [1 / 6, 2 / 3, 1 / 6],
                       [1 / 6, 1 / 6, 2 / 3]])


def quad_exact(patch):
    """The rule of the Const basis' transport terms: the accurate reference
    rule, so that M_q = |q| and A^xi_q = int_q Omega_xi to round-off (a
    reading: the paper fixes no quadrature)."""
    return quad_accurate(patch, 1)


def quad3(patch):
    """The 3-point rule of the transport terms: points at barycentric
    (2/3, 1/6, 1/6) (and permutations) of the flat triangle, mapped to the
    sphere; weights chosen so that the rule integrates the three Lin
    functions exactly (sum_k w_k psi_m(Omega_k) = int psi_m), which also
    makes the weights sum to the exact patch area."""
    omega = QUAD3_BARY @ gnomonic(patch.verts, octant_signs(patch.octant))
    omega /= np.linalg.norm(omega, axis=1)[:, None]
    om_f, w_f = quad_accurate(patch)
    exact = lin_basis(patch, om_f).T @ w_f
    psi = lin_basis(patch, omega)                     # psi[k, m] = psi_m(Omega_k)
    w = np.linalg.solve(psi.T, exact)
    return omega, w


# ------------------------------------------------------ angular matrices

class PatchRule:
    """Quadrature points, weights and basis values for a list of patches
    (Lin basis: 3 functions per patch; Const: 1)."""

    def __init__(self, patches, rule=None, basis="lin"):
        fn, self.nd = BASES[basis]
        if rule is None:
            rule = quad3 if basis == "lin" else quad_exact
        self.patches = patches
        self.omega, self.w, self.psi, self.owner = [], [], [], []
        for q, p in enumerate(patches):
            om, w = rule(p)
            self.omega.append(om)
            self.w.append(w)
            self.psi.append(fn(p, om))             # (npts, nd): psi_d(Omega_k)
            self.owner.append(np.full(len(w), q))
        self.omega = np.vstack(self.omega)
        self.w = np.concatenate(self.w)
        self.owner = np.concatenate(self.owner)

    def mass(self, q):
        """M_q[m,d] = int_{D_q} psi_m psi_d."""
        sel = self.owner == q
        ps, w = self.psi[q], self.w[sel]
        return (ps * w[:, None]).T @ ps

    def jacobian(self, q, xi):
        """A^xi_q[m,d] = int_{D_q} Omega^xi psi_m psi_d."""
        sel = self.owner == q
        ps, w, om = self.psi[q], self.w[sel], self.omega[sel, xi]
        return (ps * (w * om)[:, None]).T @ ps

    def basis_integral(self, q):
        sel = self.owner == q
        return self.psi[q].T @ self.w[sel]

    def weighted_basis(self):
        """Block matrix B (A x npts): B[(q,m), k] = w_k psi_{q,m}(Omega_k)."""
        nd = self.nd
        A, npts = nd * len(self.patches), len(self.w)
        B = np.zeros((A, npts))
        for q in range(len(self.patches)):
            idx = np.nonzero(self.owner == q)[0]
            B[nd * q:nd * q + nd, idx] = (self.psi[q] * self.w[idx][:, None]).T
        return B


def legendre_table(order, mu):
    """P_0 ... P_order at mu (Bonnet recurrence)."""
    mu = np.asarray(mu, dtype=np.float64)
    P = np.zeros((order + 1,) + mu.shape)
    P[0] = 1.0
    if order >= 1:
        P[1] = mu
    for n in range(1, order):
        P[n + 1] = ((2 * n + 1) * mu * P[n] - n * P[n - 1]) / (n + 1)
    return P


def real_harmonics(order, omega):
    """Orthonormal real spherical harmonics Y_{n,o}, n <= order, o = -n..n,
    columns ordered n^2 + n + o; built from scipy's complex harmonics."""
    from scipy.special import sph_harm_y
    omega = np.atleast_2d(omega)
    theta = np.arccos(np.clip(omega[:, 2], -1, 1))
    phi = np.arctan2(omega[:, 1], omega[:, 0])
    Y = np.zeros((len(omega), (order + 1) ** 2))
    for n in range(order + 1):
        for o in range(-n, n + 1):
            c = sph_harm_y(n, abs(o), theta, phi)
            if o == 0:
                val = c.real
            elif o > 0:
                val = math.sqrt(2.0) * (-1) ** o * c.real
            else:
                val = math.sqrt(2.0) * (-1) ** o * c.imag
            Y[:, n * n + n + o] = val
    return Y


def x_integrals(patches, order, basis="lin"):
    """X_{[q]m,no} = int_{D_q} psi_{q,m} Y_{n,o} (eq. X), shape (A, (order+1)^2),
    integrated with the accurate reference rule of each patch."""
    fn, nd = BASES[basis]
    X = np.zeros((nd * len(patches), (order + 1) ** 2))
    for q, p in enumerate(patches):
        om, w = quad_accurate(p, order)
        psi = fn(p, om)
        X[nd * q:nd * q + nd] = (psi * w[:, None]).T @ real_harmonics(order, om)
    return X


def scatter_matrix(patches, moments, basis="lin"):
    """Dense angular scatter matrix S~ (A x A) per unit sigma_s, Section 5.2:
    S~[(q,m),(p,d)] = sum_{n,o} f_n X_{[q]mno} X_{[p]dno}, with
    sigma_{s,n} = sigma_s f_n and f = ``moments`` (f_0 ... f_L)."""
    moments = np.asarray(moments, dtype=np.float64)
    L = len(moments) - 1
    X = x_integrals(patches, L, basis)
    F = np.concatenate([np.full(2 * n + 1, moments[n]) for n in range(L + 1)])
    return (X * F[None, :]) @ X.T


def scatter_matrix_addition(patches, moments, basis="lin"):
    """The same S~ through the addition theorem
    sum_o Y_no(a) Y_no(b) = (2n+1)/(4 pi) P_n(a . b): a harmonic-convention
    free cross-check (small meshes only: dense in all quadrature points)."""
    moments = np.asarray(moments, dtype=np.float64)
    L = len(moments) - 1
    rule = PatchRule(patches, lambda p: quad_accurate(p, L), basis)
    mu = np.clip(rule.omega @ rule.omega.T, -1.0, 1.0)
    P = legendre_table(L, mu)
    coef = moments * (2 * np.arange(L + 1) + 1) / (4 * math.pi)
    kern = np.tensordot(coef, P, axes=1)
    B = rule.weighted_basis()
    return B @ kern @ B.T


def scatter_rows_addition(patches, moments, q, chunk=4096, basis="lin"):
    """Rows of patch q (3q..3q+2 for Lin) of S~ through the addition theorem,
    accumulating the Legendre sum by its three-term recurrence over chunks
    of quadrature points (for meshes where the dense kernel would not fit in
    memory)."""
    fn, nd = BASES[basis]
    moments = np.asarray(moments, dtype=np.float64)
    L = len(moments) - 1
    coef = moments * (2 * np.arange(L + 1) + 1) / (4 * math.pi)
    om_q, w_q = quad_accurate(patches[q], L)
    bq = (fn(patches[q], om_q) * w_q[:, None]).T                 # (nd, nq)
    rows = np.zeros((nd, nd * len(patches)))
    for p, patch in enumerate(patches):
        om_p, w_p = quad_accurate(patch, L)
        bp = (fn(patch, om_p) * w_p[:, None]).T                 # (nd, np)
        for c0 in range(0, len(w_p), chunk):
            mu = np.clip(om_q @ om_p[c0:c0 + chunk].T, -1.0, 1.0)
            p0, p1 = np.ones_like(mu), mu
            kern = coef[0] * p0 + (coef[1] * p1 if L >= 1 else 0.0)
            for n in range(1, L):
                p0, p1 = p1, ((2 * n + 1) * mu * p1 - n * p0) / (n + 1)
                kern = kern + coef[n + 1] * p1
            rows[:, nd * p:nd * p + nd] += bq @ kern @ bp[:, c0:c0 + chunk].T
    return rows


def hg_moments(g, order):
    """Henyey-Greenstein Legendre coefficients f_n = g^n, plain truncation."""
    return np.array([g ** n for n in range(order + 1)], dtype=np.float64)


def fp_moments(alpha, N):
    """Eq. scatter_moments: sigma_{s,n} = alpha/2 (N(N+1) - n(n+1)), n <= N."""
    return np.array([0.5 * alpha * (N * (N + 1) - n * (n + 1)) for n in range(N + 1)])


# ------------------------------------------------------------ prolongation

def prolongation(coarse, fine, basis="lin"):
    """Galerkin prolongation between nested angular spaces (Section 4.1).
    Each fine patch is either a coarse patch itself or a daughter of one.
    Lin: the coarse functions are linear on the common projection plane, so
    the fine nodal coefficients are the coarse functions evaluated at the
    fine vertices.  Const: a daughter takes its parent's value.  Returns the
    dense (nd P_fine) x (nd P_coarse) matrix."""
    nd = basis_dofs(basis)
    index = {id(p): i for i, p in enumerate(coarse)}
    cut = max(p.level for p in coarse)
    P = np.zeros((nd * len(fine), nd * len(coarse)))
    for c, p in enumerate(fine):
        owner = p if id(p) in index else p.ancestor_at(cut)
        o = index[id(owner)]
        if basis == "lin":
            P[3 * c:3 * c + 3, 3 * o:3 * o + 3] = lin_basis(owner, p.verts)
        else:
            P[c, o] = 1.0
    return P
