"""Seeded synthetic hexahedral meshes (shared input generators).

These generators stand in for the paper's datasets (hex candidates built from
tetrahedral meshes, Section 7), which are not available: many independent or
vertex-sharing linear hexahedra with a valid/invalid mix.  They hold none of
the validity method's arithmetic: no Jacobian, Bezier coefficient or verdict is
computed here.  The near-degenerate generator places one corner at a chosen
height above the plane of its three neighbours (plain plane geometry).

Node order is always that of Appendix A: (0,0,0) (1,0,0) (1,1,0) (0,1,0)
(0,0,1) (1,0,1) (1,1,1) (0,1,1).
"""
import math

import numpy as np

CUBE = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                 [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.float64)

# For each corner: its neighbours along xi, eta, zeta (Appendix A numbering).
CORNER_NEIGHBOURS = np.array([[1, 3, 4], [0, 2, 5], [3, 1, 6], [2, 0, 7],
                              [5, 7, 0], [4, 6, 1], [7, 5, 2], [6, 4, 3]])


def independent_hexes(n, noise=0.35, seed=0, edge=1.0):
    """n independent hexahedra [n,8,3]: unit-cube corners scaled by `edge`,
    each corner displaced by i.i.d. uniform noise in [-noise, noise]^3."""
    rng = np.random.default_rng(seed)
    return CUBE[None] * edge + rng.uniform(-noise, noise, size=(n, 8, 3))


def lattice_vertices(nx, ny, nz, amp=0.2, wavelength=16.0, dtype=np.float64):
    """Vertices [(nx+1)(ny+1)(nz+1), 3] of a structured lattice warped by a
    smooth sinusoidal map; vertex (i,j,k) has id i + (nx+1)(j + (ny+1) k)."""
    i = np.arange(nx + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    k = np.arange(nz + 1, dtype=np.float64)
    w = 2.0 * math.pi / wavelength
    si, sj, sk = np.sin(w * i), np.sin(w * j), np.sin(w * k)
    V = np.empty((nz + 1, ny + 1, nx + 1, 3), dtype=dtype)
    V[..., 0] = i[None, None, :] + amp * (sj[None, :, None] * sk[:, None, None])
    V[..., 1] = j[None, :, None] + amp * (sk[:, None, None] * si[None, None, :])
    V[..., 2] = k[:, None, None] + amp * (si[None, None, :] * sj[None, :, None])
    return V.reshape(-1, 3)


def lattice_connectivity(nx, ny, nz):
    """int32 [nx ny nz, 8]: hex (i,j,k) -> id i + nx (j + ny k), corners in
    Appendix A order."""
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    if (nx + 1) * (ny + 1) * (nz + 1) >= 2 ** 31:
        raise ValueError("lattice too large for int32 vertex ids")
    base = (np.arange(nx, dtype=np.int32)[None, None, :]
            + sx * np.arange(ny, dtype=np.int32)[None, :, None]
            + sy * np.arange(nz, dtype=np.int32)[:, None, None]).reshape(-1)
    off = np.array([0, 1, 1 + sx, sx, sy, 1 + sy, 1 + sx + sy, sx + sy], dtype=np.int32)
    conn = np.empty((base.size, 8), dtype=np.int32)
    for c in range(8):
        conn[:, c] = base + off[c]
    return conn


def warped_lattice(nx, ny, nz, amp=0.2, wavelength=16.0, jitter_fraction=0.01, jitter=0.8,
                   seed=0, jitter_all=False):
    """A warped lattice mesh (vertices [M,3] float64, conn [N,8] int32).

    A fraction `jitter_fraction` of the vertices (chosen with
    rng.random(M) < fraction) is displaced by U(-jitter, jitter)^3 to create
    tangled elements; with jitter_all every vertex is displaced."""
    V = lattice_vertices(nx, ny, nz, amp, wavelength)
    rng = np.random.default_rng(seed)
    if jitter_all:
        V += rng.uniform(-jitter, jitter, size=V.shape)
    elif jitter_fraction > 0:
        sel = np.nonzero(rng.random(V.shape[0]) < jitter_fraction)[0]
        V[sel] += rng.uniform(-jitter, jitter, size=(sel.size, 3))
    return V, lattice_connectivity(nx, ny, nz)


def near_degenerate_hexes(n, seed=1, noise=0.15, rel=1e-7, log10_scale=3.0):
    """n independent hexahedra [n,8,3] with one corner each placed so that its
    corner tetrahedron is within `rel` (relative) of flat.

    Each hex is a unit cube plus U(-noise, noise)^3 noise.  A corner c ~ U{0..7}
    is moved to the plane of its three neighbours and then off it by
    delta * |e1| |e2| |e3| / (2 area), delta ~ U(-rel, rel), along the plane
    normal oriented towards the corner's original side.  The hex is finally
    scaled by s = 10^U(-log10_scale, log10_scale)."""
    rng = np.random.default_rng(seed)
    P = CUBE[None] + rng.uniform(-noise, noise, size=(n, 8, 3))
    c = rng.integers(0, 8, size=n)
    delta = rng.uniform(-rel, rel, size=n)
    s = 10.0 ** rng.uniform(-log10_scale, log10_scale, size=n)
    idx = np.arange(n)
    nb = CORNER_NEIGHBOURS[c]
    a, b, d = P[idx, nb[:, 0]], P[idx, nb[:, 1]], P[idx, nb[:, 2]]
    x = P[idx, c]
    normal = np.cross(b - a, d - a)
    area2 = np.linalg.norm(normal, axis=1)            # twice the triangle area
    unit = normal / area2[:, None]
    h0 = np.einsum("ij,ij->i", x - a, unit)           # signed height of the corner
    side = np.where(h0 >= 0, 1.0, -1.0)
    lengths = (np.linalg.norm(a - x, axis=1) * np.linalg.norm(b - x, axis=1)
               * np.linalg.norm(d - x, axis=1))
    h = side * delta * lengths / area2
    P[idx, c] = x - (h0 - h)[:, None] * unit
    return P * s[:, None, None]


def append_independent(V, conn, P):
    """Append independent hexahedra P [n,8,3] (8 private vertices each) to a
    shared-vertex mesh (V, conn)."""
    n = P.shape[0]
    m0 = V.shape[0]
    if m0 + 8 * n >= 2 ** 31:
        raise ValueError("too many vertices for int32 ids")
    V2 = np.concatenate([V, P.reshape(-1, 3)])
    extra = (m0 + np.arange(8 * n, dtype=np.int64)).astype(np.int32).reshape(n, 8)
    return V2, np.concatenate([conn, extra])


def precision_stress(nx=400, ny=400, nz=400, extra_fraction=0.05, seed=0, seed_extra=1):
    """The warped, 1%-tangled lattice plus `extra_fraction` x N near-degenerate
    independent hexahedra with rescaled coordinates."""
    V, conn = warped_lattice(nx, ny, nz, seed=seed)
    P = near_degenerate_hexes(int(round(extra_fraction * conn.shape[0])), seed=seed_extra)
    return append_independent(V, conn, P)


def batched_mesh_sizes(n_meshes=10000, lo=2.0, hi=6.0, seed=4):
    """Hex counts log-uniform in [10^lo, 10^hi] and lattice dimensions for each."""
    rng = np.random.default_rng(seed)
    N = np.rint(10.0 ** rng.uniform(lo, hi, size=n_meshes)).astype(np.int64)
    dims = []
    for n in N:
        nx = max(1, int(round(n ** (1.0 / 3.0))))
        nz = max(1, int(round(n / (nx * nx))))
        dims.append((nx, nx, nz))
    amps = rng.uniform(0.0, 0.6, size=n_meshes)
    return dims, amps


def batched_meshes(n_meshes=10000, lo=2.0, hi=6.0, seed=4):
    """Generator of (V, conn) for the batched workload: warped lattices with every
    vertex jittered by U(-a_m, a_m)^3, a_m ~ U(0, 0.6); mesh m uses seed
    (seed, m)."""
    dims, amps = batched_mesh_sizes(n_meshes, lo, hi, seed)
    for m, ((nx, ny, nz), a) in enumerate(zip(dims, amps)):
        V, conn = warped_lattice(nx, ny, nz, jitter=a, jitter_all=True, seed=[seed, m])
        yield V, conn


# ---------------------------------------------------------------- quadrangles

SQUARE = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float64)


def independent_quads(n, noise=0.4, seed=0):
    """n independent quadrangles [n,4,2]: unit-square corners (order (0,0)
    (1,0) (1,1) (0,1)) each displaced by U(-noise, noise)^2."""
    rng = np.random.default_rng(seed)
    return SQUARE[None] + rng.uniform(-noise, noise, size=(n, 4, 2))


def quad_lattice(nx, ny, amp=0.2, wavelength=16.0, jitter_fraction=0.01, jitter=0.8, seed=0):
    """A warped nx x ny quadrangle lattice: vertices [(nx+1)(ny+1), 2] float64
    (vertex (i,j) -> id i + (nx+1) j, x = i + amp sin(2 pi j / wavelength),
    y = j + amp sin(2 pi i / wavelength)), a fraction of them displaced by
    U(-jitter, jitter)^2, and connectivity [nx ny, 4] int32 (quad (i,j) -> id
    i + nx j, corners (i,j) (i+1,j) (i+1,j+1) (i,j+1))."""
    w = 2.0 * math.pi / wavelength
    i = np.arange(nx + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    V = np.empty((ny + 1, nx + 1, 2), dtype=np.float64)
    V[..., 0] = i[None, :] + amp * np.sin(w * j)[:, None]
    V[..., 1] = j[:, None] + amp * np.sin(w * i)[None, :]
    V = V.reshape(-1, 2)
    rng = np.random.default_rng(seed)
    if jitter_fraction > 0:
        sel = np.nonzero(rng.random(V.shape[0]) < jitter_fraction)[0]
        V[sel] += rng.uniform(-jitter, jitter, size=(sel.size, 2))
    sx = nx + 1
    if (nx + 1) * (ny + 1) >= 2 ** 31:
        raise ValueError("lattice too large for int32 vertex ids")
    base = (np.arange(nx, dtype=np.int32)[None, :] + sx * np.arange(ny, dtype=np.int32)[:, None]).reshape(-1)
    C = np.empty((base.size, 4), dtype=np.int32)
    for k, off in enumerate((0, 1, 1 + sx, sx)):
        C[:, k] = base + off
    return V, C


# ---------------------------------------------------------------- on device

def warped_lattice_torch(nx, ny, nz, amp=0.2, wavelength=16.0, jitter=0.0, seed=0, device="cuda"):
    """warped_lattice generated on the device with torch (every vertex jittered
    by U(-jitter, jitter)^3 from a Philox stream seeded with `seed`).  Returns
    (vertices float64 [M,3], connectivity int32 [N,8]) device tensors."""
    import torch
    w = 2.0 * math.pi / wavelength
    i = torch.arange(nx + 1, dtype=torch.float64, device=device)
    j = torch.arange(ny + 1, dtype=torch.float64, device=device)
    k = torch.arange(nz + 1, dtype=torch.float64, device=device)
    si, sj, sk = torch.sin(w * i), torch.sin(w * j), torch.sin(w * k)
    V = torch.empty((nz + 1, ny + 1, nx + 1, 3), dtype=torch.float64, device=device)
    V[..., 0] = i[None, None, :] + amp * (sj[None, :, None] * sk[:, None, None])
    V[..., 1] = j[None, :, None] + amp * (sk[:, None, None] * si[None, None, :])
    V[..., 2] = k[:, None, None] + amp * (si[None, None, :] * sj[None, :, None])
    V = V.reshape(-1, 3)
    if jitter > 0:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed))
        V += (torch.rand(V.shape, dtype=torch.float64, device=device, generator=g) * 2.0 - 1.0) * jitter
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    base = (torch.arange(nx, dtype=torch.int32, device=device)[None, None, :]
            + sx * torch.arange(ny, dtype=torch.int32, device=device)[None, :, None]
            + sy * torch.arange(nz, dtype=torch.int32, device=device)[:, None, None]).reshape(-1, 1)
    off = torch.tensor([0, 1, 1 + sx, sx, sy, 1 + sy, 1 + sx + sy, sx + sy], dtype=torch.int32,
                       device=device)
    return V, (base + off[None, :]).contiguous()


def batched_meshes_torch(n_meshes=10000, lo=2.0, hi=6.0, seed=4, device="cuda"):
    """The batched workload on the device: mesh m is a warped lattice with
    every vertex jittered by U(-a_m, a_m)^3, a_m ~ U(0, 0.6), hex counts
    log-uniform in [10^lo, 10^hi] (dimensions from batched_mesh_sizes).
    Yields (V, conn) device tensors; jitter stream of mesh m seeded seed*1e6+m."""
    dims, amps = batched_mesh_sizes(n_meshes, lo, hi, seed)
    for m, ((nx, ny, nz), a) in enumerate(zip(dims, amps)):
        yield warped_lattice_torch(nx, ny, nz, jitter=float(a), seed=seed * 1_000_000 + m,
                                   device=device)


def near_degenerate_mesh_torch(n_lattice_cells, seed=0, device="cuda"):
    """A serving request mesh generated as in the precision-stress workload:
    a warped lattice of about n cells (1% of vertices jittered 0.8) plus 5%
    near-degenerate independent hexes; lattice on the device, the appended
    hexes from near_degenerate_hexes (host) copied over."""
    import torch
    n = max(1, int(n_lattice_cells))
    nx = max(1, int(round(n ** (1.0 / 3.0))))
    nz = max(1, int(round(n / (nx * nx))))
    V, C = warped_lattice_torch(nx, nx, nz, seed=seed, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + 7)
    sel = torch.rand(V.shape[0], dtype=torch.float64, device=device, generator=g) < 0.01
    V[sel] += (torch.rand((int(sel.sum()), 3), dtype=torch.float64, device=device, generator=g) * 2 - 1) * 0.8
    n_extra = int(round(0.05 * C.shape[0]))
    if n_extra:
        P = torch.from_numpy(near_degenerate_hexes(n_extra, seed=int(seed) + 11)).to(device)
        extra = (V.shape[0] + torch.arange(8 * n_extra, dtype=torch.int64, device=device)).to(
            torch.int32).reshape(n_extra, 8)
        V = torch.cat([V, P.reshape(-1, 3)])
        C = torch.cat([C, extra])
    return V.contiguous(), C.contiguous()
