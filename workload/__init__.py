"""Seeded synthetic inputs shared by the oracle and the GPU library.

This module only *generates input data* (meshes, partitions, coefficient
fields, right-hand-side sequences).  It holds none of the solver's arithmetic:
no stiffness matrices, no substructuring, no preconditioner, no Krylov method.
Both the CPU oracle (``oracle/``) and the HIP path (``paper_2412_17543_amd``)
consume what it returns, the way they would both read the same input file.

Conventions (used by every consumer):

* structured box of ``nx*ny*nz`` hexahedral elements on the unit cube,
  element size ``h = 1/nx``;
* node ``(ix, iy, iz)`` has index ``ix + (nx+1)*(iy + (ny+1)*iz)``
  (x fastest), element ``(ex, ey, ez)`` has index ``ex + nx*(ey + ny*ez)``;
* element vertex ``v = a + 2b + 4c`` sits at offset ``(a, b, c)``.

Seeds come from one root ``SeedSequence`` split per purpose, so that e.g. the
noise of step k never changes when the number of steps changes.

The right-hand side of the pressure-corrector problem (Section 2, eq. of the
algebraic systems) changes every time step while the matrix is fixed; the paper's
sequence comes from a flow solver that is not available, so a drifting sum of
Gaussians with additive noise stands in for it (the paper only fixes "fixed SPD
matrix, new right-hand side each step").
"""
from __future__ import annotations

import numpy as np

ROOT_SEED = 20241217
PURPOSES = ("centres", "directions", "noise", "coef", "partition", "target", "fd", "misc")


def seed(purpose: str) -> np.random.SeedSequence:
    """Per-purpose child of the root seed sequence."""
    kids = np.random.SeedSequence(ROOT_SEED).spawn(len(PURPOSES))
    return kids[PURPOSES.index(purpose)]


def rng(purpose: str, *sub: int) -> np.random.Generator:
    ss = seed(purpose)
    for s in sub:
        ss = ss.spawn(s + 1)[s]
    return np.random.default_rng(ss)


# ----------------------------------------------------------------------------
# mesh index helpers (pure bookkeeping)
# ----------------------------------------------------------------------------

def n_nodes(nx: int, ny: int | None = None, nz: int | None = None) -> int:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return (nx + 1) * (ny + 1) * (nz + 1)


def element_nodes(nx: int, ny: int | None = None, nz: int | None = None) -> np.ndarray:
    """(n_elem, 8) int64 array of node indices, vertex v = a + 2b + 4c."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    e = np.arange(nx * ny * nz, dtype=np.int64)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    out = np.empty((e.size, 8), dtype=np.int64)
    for v in range(8):
        a, b, c = v & 1, (v >> 1) & 1, (v >> 2) & 1
        out[:, v] = (ex + a) + (nx + 1) * ((ey + b) + (ny + 1) * (ez + c))
    return out


def node_coords(nx: int, ny: int | None = None, nz: int | None = None) -> np.ndarray:
    """(n_nodes, 3) coordinates, h = 1/nx in every direction."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    h = 1.0 / nx
    n = np.arange((nx + 1) * (ny + 1) * (nz + 1), dtype=np.int64)
    ix, iy, iz = n % (nx + 1), (n // (nx + 1)) % (ny + 1), n // ((nx + 1) * (ny + 1))
    return np.stack([ix * h, iy * h, iz * h], axis=1)


def element_centroids(nx: int) -> np.ndarray:
    h = 1.0 / nx
    e = np.arange(nx ** 3, dtype=np.int64)
    ex, ey, ez = e % nx, (e // nx) % nx, e // (nx * nx)
    return np.stack([(ex + 0.5) * h, (ey + 0.5) * h, (ez + 0.5) * h], axis=1)


# ----------------------------------------------------------------------------
# partitions (element -> subdomain, subdomain -> subregion)
# ----------------------------------------------------------------------------

def cube_partition(nx: int, sub_elems: int) -> np.ndarray:
    """Split an nx^3 box into (nx/sub_elems)^3 cube subdomains, lexicographic."""
    assert nx % sub_elems == 0
    m = nx // sub_elems
    e = np.arange(nx ** 3)
    ex, ey, ez = e % nx, (e // nx) % nx, e // (nx * nx)
    sx, sy, sz = ex // sub_elems, ey // sub_elems, ez // sub_elems
    return (sx + m * (sy + m * sz)).astype(np.int32)


def cube_subregions(m: int, group: int) -> np.ndarray:
    """Group an m^3 lattice of subdomains into (m/group)^3 subregions."""
    assert m % group == 0
    g = m // group
    s = np.arange(m ** 3)
    sx, sy, sz = s % m, (s // m) % m, s // (m * m)
    return ((sx // group) + g * ((sy // group) + g * (sz // group))).astype(np.int32)


def sphere_hole_keep(nx: int, centre=(0.5, 0.5, 0.5), radius: float = 0.15) -> np.ndarray:
    """uint8 mask: 1 for elements kept, 0 for elements whose centroid lies in the ball."""
    c = element_centroids(nx)
    d2 = ((c - np.asarray(centre)) ** 2).sum(axis=1)
    return (d2 > radius * radius).astype(np.uint8)


def _rcb_split(points: np.ndarray, ids: np.ndarray, k: int, g: np.random.Generator, lo: float, hi: float,
               out: np.ndarray, first: int) -> int:
    """Assign parts first..first+k-1 to ids by recursive coordinate bisection:
    cut along the longest extent, a fraction f ~ U[lo, hi] of the points to
    the first floor(k/2) parts (f = 1/2 when lo == hi == 0.5)."""
    if k == 1:
        out[ids] = first
        return first + 1
    p = points[ids]
    axis = int(np.argmax(p.max(axis=0) - p.min(axis=0)))
    order = np.argsort(p[:, axis], kind="stable")
    k1 = k // 2
    f = g.uniform(lo, hi) if hi > lo else lo
    if lo == hi == 0.5:
        f = k1 / k
    cut = min(max(int(round(f * len(ids))), 1), len(ids) - 1)
    nxt = _rcb_split(points, ids[order[:cut]], k1, g, lo, hi, out, first)
    return _rcb_split(points, ids[order[cut:]], k - k1, g, lo, hi, out, nxt)


def _face_components(nx: int, part: np.ndarray, keep: np.ndarray) -> np.ndarray:
    """Label connected components (through shared element faces) of each part;
    returns a new part id per element (removed elements: -1)."""
    n = nx ** 3
    par = np.arange(n)

    def find(a):
        while par[a] != a:
            par[a] = par[par[a]]
            a = par[a]
        return a

    e = np.arange(n)
    ex, ey, ez = e % nx, (e // nx) % nx, e // (nx * nx)
    for d, ok in ((1, ex < nx - 1), (nx, ey < nx - 1), (nx * nx, ez < nx - 1)):
        a = e[ok]
        b = a + d
        same = keep[a].astype(bool) & keep[b].astype(bool) & (part[a] == part[b])
        for u, v in zip(a[same], b[same]):
            ru, rv = find(u), find(v)
            if ru != rv:
                par[max(ru, rv)] = min(ru, rv)
    roots = np.array([find(x) for x in range(n)])
    lab = np.full(n, -1, dtype=np.int64)
    kept = keep.astype(bool)
    _, inv = np.unique(roots[kept], return_inverse=True)
    lab[kept] = inv
    return lab


def interior_counts(nx: int, part: np.ndarray, keep: np.ndarray) -> np.ndarray:
    """Interior free nodes per part: nodes touched by elements of that part
    only, excluding the Dirichlet face x = 1."""
    en = element_nodes(nx)[keep.astype(bool)]
    pe = part[keep.astype(bool)]
    nn = n_nodes(nx)
    first = np.full(nn, -1, dtype=np.int64)
    multi = np.zeros(nn, dtype=bool)
    for v in range(8):
        nd = en[:, v]
        unset = first[nd] < 0
        first[nd[unset]] = pe[unset]
        multi[nd[(~unset) & (first[nd] != pe)]] = True
    # a second pass catches nodes first set by a later element of another part
    for v in range(8):
        nd = en[:, v]
        multi[nd[first[nd] != pe]] = True
    dirichlet = (np.arange(nn) % (nx + 1)) == nx
    ok = (first >= 0) & ~multi & ~dirichlet
    return np.bincount(first[ok], minlength=int(part.max()) + 1)


def rcb_partition(nx: int, n_parts: int, keep: np.ndarray | None = None, lo: float = 0.3, hi: float = 0.7,
                  min_interior: int = 0, sub: int = 0) -> np.ndarray:
    """Seeded jittered recursive coordinate bisection of the kept elements into
    n_parts face-connected subdomains (removed elements get part 0).

    Cuts take a fraction f ~ U[lo, hi] of the points; disconnected pieces are
    split into their own parts, then the part with the fewest interior free
    nodes is merged into the face neighbour sharing most faces with it until
    n_parts remain and every part has at least min_interior interior nodes
    (or no merge is possible)."""
    keep = np.ones(nx ** 3, dtype=np.uint8) if keep is None else keep
    kept = np.nonzero(keep)[0]
    out = np.zeros(nx ** 3, dtype=np.int64)
    _rcb_split(element_centroids(nx), kept, n_parts, rng("partition", sub), lo, hi, out, 0)
    part = _face_components(nx, out, keep)
    e = np.arange(nx ** 3)
    ex, ey, ez = e % nx, (e // nx) % nx, e // (nx * nx)
    pairs = []
    for d, ok in ((1, ex < nx - 1), (nx, ey < nx - 1), (nx * nx, ez < nx - 1)):
        a = e[ok]
        b = a + d
        m = keep[a].astype(bool) & keep[b].astype(bool)
        pairs.append((a[m], b[m]))
    while True:
        npart = int(part.max()) + 1
        cnt = interior_counts(nx, part, keep)
        if npart <= n_parts and cnt.min() >= min_interior:
            break
        if npart <= 1:
            break
        small = int(np.argmin(cnt))
        shared = np.zeros(npart, dtype=np.int64)
        for a, b in pairs:
            pa, pb = part[a], part[b]
            m = (pa == small) & (pb != small)
            np.add.at(shared, pb[m], 1)
            m = (pb == small) & (pa != small)
            np.add.at(shared, pa[m], 1)
        if shared.max() == 0:
            break
        tgt = int(np.argmax(shared))
        part[part == small] = tgt
        part[part > small] -= 1
    part[~keep.astype(bool)] = 0
    return part.astype(np.int32)


def rcb_subregions(nx: int, part: np.ndarray, keep: np.ndarray, n_groups: int) -> np.ndarray:
    """Group subdomains into n_groups subregions of (nearly) equal count by
    recursive coordinate bisection of the subdomain centroids."""
    c = element_centroids(nx)[keep.astype(bool)]
    p = part[keep.astype(bool)]
    n = int(p.max()) + 1
    cen = np.stack([np.bincount(p, weights=c[:, d], minlength=n) for d in range(3)], axis=1)
    cen /= np.bincount(p, minlength=n)[:, None]
    out = np.zeros(n, dtype=np.int64)
    _rcb_split(cen, np.arange(n), n_groups, rng("partition", 99), 0.5, 0.5, out, 0)
    return out.astype(np.int32)


def lognormal_coef(n_elem: int, sigma: float, purpose: str = "coef", sub: int = 0) -> np.ndarray:
    """Per-element coefficient exp(sigma * xi), xi ~ N(0, 1)."""
    g = rng(purpose, sub)
    return np.exp(sigma * g.standard_normal(n_elem))


# ----------------------------------------------------------------------------
# right-hand-side sequence
# ----------------------------------------------------------------------------

def _reflect01(x: np.ndarray) -> np.ndarray:
    """Reflect coordinates back into [0, 1] (mirror at the box faces)."""
    y = np.mod(x, 2.0)
    return np.where(y > 1.0, 2.0 - y, y)


def gaussian_centres(n_rhs: int, n_gauss: int = 4, drift: float = 0.01) -> np.ndarray:
    """(n_rhs, n_gauss, 3) drifting centres c_{g,k} = c_{g,0} + drift*k*d_g, reflected."""
    c0 = rng("centres").uniform(0.2, 0.8, size=(n_gauss, 3))
    d = rng("directions").standard_normal((n_gauss, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    k = np.arange(n_rhs)[:, None, None]
    return _reflect01(c0[None] + drift * k * d[None])


def nodal_source(nx: int, k: int, centres: np.ndarray, width: float = 0.1,
                 noise: float = 1e-3) -> np.ndarray:
    """Nodal values of f_k = sum_g exp(-|x-c|^2/(2 w^2)) + noise * N(0,1) on the
    (nx+1)^3 grid of the unit cube.  Each Gaussian is the product of three
    one-dimensional factors, formed as an outer product."""
    t = np.arange(nx + 1) / nx
    f = np.zeros((nx + 1, nx + 1, nx + 1))                 # (z, y, x), x fastest
    for c in centres[k]:
        g = [np.exp(-((t - c[d]) ** 2) / (2.0 * width * width)) for d in range(3)]
        f += g[2][:, None, None] * (g[1][None, :, None] * g[0][None, None, :])
    f = f.ravel()
    f += noise * rng("noise", k).standard_normal(f.size)
    return f


_M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


def _mass_1d(v: np.ndarray, axis: int) -> np.ndarray:
    """Apply the assembled one-dimensional mass matrix (unit spacing: 2/3 on
    the diagonal, 1/3 at both ends, 1/6 beside it) along one axis."""
    v = np.moveaxis(v, axis, 0)
    out = v * (2.0 / 3.0)
    out[0] = v[0] / 3.0
    out[-1] = v[-1] / 3.0
    out[1:] += v[:-1] / 6.0
    out[:-1] += v[1:] / 6.0
    return np.moveaxis(out, 0, axis)


def consistent_load(nx: int, f_nodal: np.ndarray, elem_keep: np.ndarray | None = None) -> np.ndarray:
    """Load vector F = M f of trilinear interpolant f with the consistent Q1 mass.

    This is input preparation (turning a nodal source into a load vector), the
    same for every consumer; M_e = h^3 (M1 (x) M1 (x) M1).  On the whole box the
    assembled M is the Kronecker product of three one-dimensional mass
    matrices and is applied axis by axis; with removed elements it is
    assembled element by element.
    """
    h = 1.0 / nx
    if elem_keep is None:
        v = f_nodal.reshape(nx + 1, nx + 1, nx + 1)
        for axis in range(3):
            v = _mass_1d(v, axis)
        return (v * h ** 3).ravel()
    mref = np.kron(_M1, np.kron(_M1, _M1)) * h ** 3  # vertex v = a + 2b + 4c, x fastest
    en = element_nodes(nx)[elem_keep.astype(bool)]
    fe = f_nodal[en] @ mref.T
    return np.bincount(en.ravel(), weights=fe.ravel(), minlength=n_nodes(nx))


def rhs_sequence(nx: int, n_rhs: int, elem_keep: np.ndarray | None = None,
                 first: int = 0) -> np.ndarray:
    """(n_rhs, n_nodes) float64 load vectors F_k, k = first .. first+n_rhs-1."""
    cen = gaussian_centres(first + n_rhs)
    out = np.empty((n_rhs, n_nodes(nx)))
    for i in range(n_rhs):
        out[i] = consistent_load(nx, nodal_source(nx, first + i, cen), elem_keep)
    return out


def consistent_neumann(nx: int, F: np.ndarray, elem_keep: np.ndarray | None = None) -> np.ndarray:
    """Load vectors made consistent for the pure Neumann problem (no Dirichlet
    node: K has the constants as null space, so F must sum to zero): the
    source is shifted by a constant, F - c M 1, with c = sum(F) / sum(M 1)."""
    m = consistent_load(nx, np.ones(n_nodes(nx)), elem_keep)
    F = np.atleast_2d(F)
    return F - np.outer(F.sum(axis=1) / m.sum(), m)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def workload(name: str) -> dict:
    """Mesh/partition/options of the named synthetic workloads.

    * ``c16``: 16^3 elements, 2x2x2 subdomains of 8^3, two-level, plain PCG, 10 RHS.
    * ``c64``: 64^3 elements, 8^3 subdomains of 8^3, three-level (subregions of
      2x2x2 subdomains), deflated PCG with a 20-vector recycled basis, 50 RHS.
    * ``c96``: 96^3 elements, 12^3 subdomains, three-level, 20 RHS (adjoint form).
    * ``c192``: 192^3 elements, 24^3 subdomains, three-level, 40-vector basis.
    * ``tiny``: 8^3 elements, 2x2x2 subdomains of 4^3 (tests).
    * ``c3``: 64^3 box with a spherical hole (radius 0.15, centre 0.5), seeded
      jittered RCB into 400 face-connected subdomains of uneven size, 50
      subregions of 8 by RCB, log-normal coefficients (sigma 0.5), R = 20,
      50 right-hand sides.
    * ``c3s``: the same construction at 24^3 with 24 subdomains in 3
      subregions (parity-test size).
    * ``c16n``, ``tiny3n``: ``c16`` and ``tiny3`` without Dirichlet nodes (the
      pure Neumann problem; ``node_dirichlet`` all zero, right-hand sides made
      consistent with ``consistent_neumann``).
    """
    specs = {
        "tiny": dict(nx=8, sub=4, group=0, R=0, n_rhs=3),
        "tiny3": dict(nx=16, sub=4, group=2, R=0, n_rhs=3),
        "c16": dict(nx=16, sub=8, group=0, R=0, n_rhs=10),
        "c64": dict(nx=64, sub=8, group=2, R=20, n_rhs=50),
        "c96": dict(nx=96, sub=8, group=2, R=20, n_rhs=20),
        "c192": dict(nx=192, sub=8, group=2, R=40, n_rhs=200),
    }
    if name in ("c3", "c3s"):
        return _hole_workload(name)
    neumann = name.endswith("n") and name[:-1] in specs
    s = dict(specs[name[:-1] if neumann else name])
    nx, sub, group = s["nx"], s["sub"], s["group"]
    m = nx // sub
    s["elem_to_sub"] = cube_partition(nx, sub)
    s["n_sub"] = m ** 3
    if group:
        s["sub_to_subregion"] = cube_subregions(m, group)
        s["n_subregion"] = (m // group) ** 3
    else:
        s["sub_to_subregion"] = None
        s["n_subregion"] = 0
    s["coef"] = np.ones(nx ** 3)
    s["elem_keep"] = None
    s["name"] = name
    s["node_dirichlet"] = np.zeros(n_nodes(nx), dtype=np.uint8) if neumann else None
    return s


def _hole_workload(name: str) -> dict:
    """Uneven-batching workload: hole, jittered RCB partition, log-normal coefficients."""
    if name == "c3":
        nx, n_sub, n_sr, min_int, n_rhs = 64, 400, 50, 0, 50
    else:
        nx, n_sub, n_sr, min_int, n_rhs = 24, 24, 3, 0, 3
    keep = sphere_hole_keep(nx)
    part = rcb_partition(nx, n_sub, keep, 0.3, 0.7, min_int)
    s = dict(nx=nx, R=20, n_rhs=n_rhs, name=name, elem_keep=keep, elem_to_sub=part)
    s["n_sub"] = int(part[keep.astype(bool)].max()) + 1
    s["sub_to_subregion"] = rcb_subregions(nx, part, keep, n_sr)
    s["n_subregion"] = n_sr
    s["coef"] = lognormal_coef(nx ** 3, 0.5)
    s["node_dirichlet"] = None
    return s
