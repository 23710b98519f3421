"""Seeded synthetic workloads for the geometry stage.

This module only builds inputs: indexed triangle meshes (uint32 index
buffer, 8-float AoS vertex buffer), triangle orders, and the host-side
shader parameters (matrices, lights) that a draw is shaded with.  It holds
none of the vertex-reuse arithmetic: no batching, no deduplication and no
shading happen here.  Both the oracle tests and the GPU path take their
inputs from these generators so that they see identical bytes.

Random numbers come from SplitMix64 used as a counter-based generator:
draw i of a stream is the SplitMix64 output for state ``base + (i+1)*gamma``
where ``base`` mixes the seed and a per-purpose tag.  Uniform floats use the
top 24 bits of a draw (exactly representable in float32 and float64).

The paper evaluates on scanned models and game captures that are not
available here (Section 4); these generators stand in for them:
icospheres for closed scanned meshes (ideal reuse 5/6 as for the closed
models of Table 1), Hilbert order with local swaps for a locality-optimised
order, a full random permutation for an unoptimised order, and jittered
grids for regular patches.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

VERTEX_FLOATS = 8          # px py pz nx ny nz u v
MAX_LIGHTS = 16

SHADER_MVP = 0
SHADER_PHONG = 1
SHADER_OFFSET = 2


# --------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood 2014), counter based
# --------------------------------------------------------------------------
def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def u64_stream(seed: int, tag: int, n: int) -> np.ndarray:
    """n SplitMix64 draws for (seed, tag)."""
    with np.errstate(over="ignore"):
        base = _mix(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
                    ^ _mix(np.array([tag & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64) * _GAMMA))
        ctr = np.arange(1, n + 1, dtype=np.uint64)
        return _mix(base + ctr * _GAMMA)


def uniform(seed: int, tag: int, n: int) -> np.ndarray:
    """n uniform floats in [0, 1) with 24-bit resolution (float64 array)."""
    return (u64_stream(seed, tag, n) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


# --------------------------------------------------------------------------
# Space-filling-curve keys
# --------------------------------------------------------------------------
def hilbert2d(x: np.ndarray, y: np.ndarray, order_bits: int) -> np.ndarray:
    """Distance along the 2D Hilbert curve of cells (x, y) on a 2^b grid."""
    n = 1 << order_bits
    x = x.astype(np.int64).copy()
    y = y.astype(np.int64).copy()
    d = np.zeros_like(x)
    s = n >> 1
    while s > 0:
        rx = ((x & s) > 0).astype(np.int64)
        ry = ((y & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        # rotate the quadrant
        flip = (ry == 0) & (rx == 1)
        x = np.where(flip, n - 1 - x, x)
        y = np.where(flip, n - 1 - y, y)
        swap = ry == 0
        x, y = np.where(swap, y, x), np.where(swap, x, y)
        s >>= 1
    return d


def hilbert3d(q: np.ndarray, bits: int) -> np.ndarray:
    """Hilbert key of integer points q (n, 3) with `bits` bits per axis.

    Transpose form of Skilling, "Programming the Hilbert curve" (2004),
    followed by bit interleaving.
    """
    X = q.astype(np.int64).copy()
    M = 1 << (bits - 1)
    Q = M
    while Q > 1:
        P = Q - 1
        for i in range(3):
            hit = (X[:, i] & Q) != 0
            X[:, 0] = np.where(hit, X[:, 0] ^ P, X[:, 0])
            t = np.where(hit, 0, (X[:, 0] ^ X[:, i]) & P)
            X[:, 0] ^= t
            X[:, i] ^= t
        Q >>= 1
    X[:, 1] ^= X[:, 0]
    X[:, 2] ^= X[:, 1]
    t = np.zeros(len(X), dtype=np.int64)
    Q = M
    while Q > 1:
        t = np.where((X[:, 2] & Q) != 0, t ^ (Q - 1), t)
        Q >>= 1
    X ^= t[:, None]
    key = np.zeros(len(X), dtype=np.int64)
    for b in range(bits - 1, -1, -1):
        for i in range(3):
            key = (key << 1) | ((X[:, i] >> b) & 1)
    return key


# --------------------------------------------------------------------------
# Meshes
# --------------------------------------------------------------------------
@dataclass
class Mesh:
    name: str
    indices: np.ndarray        # uint32 [3T]
    vertices: np.ndarray       # float32 [V, 8]
    meta: dict = field(default_factory=dict)

    @property
    def num_tris(self) -> int:
        return len(self.indices) // 3

    @property
    def num_verts(self) -> int:
        return self.vertices.shape[0]


def _grid_cells(nx: int, ny: int):
    ci, cj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    return ci.ravel(), cj.ravel()          # row-major cells: j outer, i inner


def grid_mesh(nx: int, ny: int, seed: int, order: str = "scan") -> Mesh:
    """Jittered nx-by-ny vertex grid on a gentle height field.

    Vertex (i, j) has id j*nx + i.  Cell (i, j) gives the triangles
    (v(i,j), v(i+1,j), v(i+1,j+1)) and (v(i,j), v(i+1,j+1), v(i,j+1)); the two
    triangles of a cell stay adjacent in every order.
    """
    assert nx >= 2 and ny >= 2
    V = nx * ny
    j, i = np.divmod(np.arange(V, dtype=np.int64), nx)
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    jit = uniform(seed, 1, 2 * V).reshape(V, 2) * 0.2 - 0.1
    x = (i + jit[:, 0]) * hx
    y = (j + jit[:, 1]) * hy
    amp, fx, fy = 0.05, 1.5, 1.0
    z = amp * np.sin(2 * np.pi * fx * x) * np.cos(2 * np.pi * fy * y)
    dzdx = amp * 2 * np.pi * fx * np.cos(2 * np.pi * fx * x) * np.cos(2 * np.pi * fy * y)
    dzdy = -amp * 2 * np.pi * fy * np.sin(2 * np.pi * fx * x) * np.sin(2 * np.pi * fy * y)
    n = np.stack([-dzdx, -dzdy, np.ones_like(x)], axis=1)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    vert = np.empty((V, VERTEX_FLOATS), dtype=np.float64)
    vert[:, 0], vert[:, 1], vert[:, 2] = x, y, z
    vert[:, 3:6] = n
    vert[:, 6] = i * hx
    vert[:, 7] = j * hy

    ci, cj = _grid_cells(nx, ny)
    v00 = cj * nx + ci
    v10 = v00 + 1
    v11 = v00 + nx + 1
    v01 = v00 + nx
    C = len(ci)
    if order == "scan":
        cperm = np.arange(C)
    elif order == "hilbert":
        bits = max(1, int(math.ceil(math.log2(max(nx - 1, ny - 1)))))
        cperm = np.argsort(hilbert2d(ci, cj, bits), kind="stable")
    elif order == "random":
        cperm = None
    else:
        raise ValueError(order)
    tris = np.empty((C, 2, 3), dtype=np.int64)
    tris[:, 0] = np.stack([v00, v10, v11], axis=1)
    tris[:, 1] = np.stack([v00, v11, v01], axis=1)
    if cperm is not None:
        tris = tris[cperm].reshape(-1, 3)
    else:
        tris = tris.reshape(-1, 3)
        tris = tris[random_permutation(len(tris), seed, 7)]
    return Mesh(f"grid{nx}x{ny}_{order}", tris.astype(np.uint32).ravel(),
                vert.astype(np.float32), {"kind": "grid", "nx": nx, "ny": ny, "order": order,
                                          "seed": seed})


def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    P = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            P += [(a, b, 0.0), (0.0, a, b), (b, 0.0, a)]
    P = np.array(P, dtype=np.float64)
    # faces: triples whose pairwise distances all equal the edge length 2
    D = np.linalg.norm(P[:, None, :] - P[None, :, :], axis=2)
    adj = np.abs(D - 2.0) < 1e-9
    F = []
    for a in range(12):
        for b in range(a + 1, 12):
            for c in range(b + 1, 12):
                if adj[a, b] and adj[b, c] and adj[a, c]:
                    nrm = np.cross(P[b] - P[a], P[c] - P[a])
                    F.append((a, b, c) if nrm @ (P[a] + P[b] + P[c]) > 0 else (a, c, b))
    assert len(F) == 20
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    return P, np.array(F, dtype=np.int64)


def icosphere_mesh(level: int, seed: int, order: str = "scan",
                   swap_frac: float = 0.0, swap_window: int = 256) -> Mesh:
    """Unit icosphere after `level` midpoint subdivisions (V = 10*4^k + 2,
    T = 20*4^k).  Generation ("scan") order: triangle t of level k-1 becomes
    triangles 4t..4t+3 of level k; midpoint vertices are appended in
    ascending (min, max) edge-key order."""
    P, F = _icosahedron()
    for _ in range(level):
        V = len(P)
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
        e.sort(axis=1)
        key = e[:, 0] * V + e[:, 1]
        ukey, inv = np.unique(key, return_inverse=True)
        a, b = np.divmod(ukey, V)
        mid = P[a] + P[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        P = np.concatenate([P, mid])
        Tn = len(F)
        mab = V + inv[:Tn]
        mbc = V + inv[Tn:2 * Tn]
        mca = V + inv[2 * Tn:]
        A, B, C = F[:, 0], F[:, 1], F[:, 2]
        F = np.stack([np.stack([A, mab, mca], 1), np.stack([mab, B, mbc], 1),
                      np.stack([mca, mbc, C], 1), np.stack([mab, mbc, mca], 1)], axis=1).reshape(-1, 3)
    Vn = len(P)
    vert = np.empty((Vn, VERTEX_FLOATS), dtype=np.float64)
    vert[:, 0:3] = P
    vert[:, 3:6] = P
    vert[:, 6] = np.arctan2(P[:, 1], P[:, 0]) / (2 * np.pi) + 0.5
    vert[:, 7] = np.arccos(np.clip(P[:, 2], -1.0, 1.0)) / np.pi
    T = len(F)
    if order == "scan":
        perm = np.arange(T)
    elif order == "hilbert":
        cen = P[F].mean(axis=1)
        qz = np.clip(np.floor((cen + 1.0) * 0.5 * 1024.0), 0, 1023).astype(np.int64)
        k = hilbert3d(qz, 10)
        perm = np.lexsort((np.arange(T), k))     # ties broken by triangle id
    elif order == "random":
        perm = random_permutation(T, seed, 7)
    else:
        raise ValueError(order)
    if swap_frac > 0.0:
        perm = local_swaps(perm, swap_frac, swap_window, seed)
    F = F[perm]
    name = f"icosphere{level}_{order}" + (f"_swap{int(round(swap_frac * 100))}" if swap_frac else "")
    return Mesh(name, F.astype(np.uint32).ravel(), vert.astype(np.float32),
                {"kind": "icosphere", "level": level, "order": order, "swap_frac": swap_frac,
                 "seed": seed})


def random_permutation(n: int, seed: int, tag: int) -> np.ndarray:
    """Seeded permutation of range(n): stable argsort of SplitMix64 draws."""
    return np.argsort(u64_stream(seed, tag, n), kind="stable")


def local_swaps(perm: np.ndarray, frac: float, window: int, seed: int) -> np.ndarray:
    """For every window of `window` consecutive entries, visit positions in
    order; position i swaps with a uniform position j of the same window
    when its draw is below `frac`."""
    perm = perm.copy()
    n = len(perm)
    nw = (n + window - 1) // window
    u = uniform(seed, 11, nw * window).reshape(nw, window)
    w = uniform(seed, 12, nw * window).reshape(nw, window)
    starts = np.arange(nw) * window
    lens = np.minimum(window, n - starts)
    for i in range(window):
        live = (i < lens) & (u[:, i] < frac)
        if not live.any():
            continue
        src = starts[live] + i
        dst = starts[live] + np.minimum((w[live, i] * lens[live]).astype(np.int64), lens[live] - 1)
        tmp = perm[src].copy()
        perm[src] = perm[dst]
        perm[dst] = tmp
    return perm


def take_prefix(mesh: Mesh, num_tris: int) -> Mesh:
    """The draw of the first num_tris triangles of a mesh (vertex buffer
    unchanged, so some vertices may be unreferenced)."""
    return Mesh(f"{mesh.name}[:{num_tris}]", mesh.indices[:3 * num_tris].copy(), mesh.vertices,
                dict(mesh.meta, prefix=num_tris))


# --------------------------------------------------------------------------
# Shader parameters (host-side inputs, built in float64, stored as float32)
# --------------------------------------------------------------------------
def _perspective(fovy_deg, aspect, znear, zfar):
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    M = np.zeros((4, 4))
    M[0, 0] = f / aspect
    M[1, 1] = f
    M[2, 2] = (zfar + znear) / (znear - zfar)
    M[2, 3] = 2.0 * zfar * znear / (znear - zfar)
    M[3, 2] = -1.0
    return M


def _look_at(eye, target, up):
    f = target - eye
    f /= np.linalg.norm(f)
    if abs(f @ up) > 0.99:
        up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    s = np.cross(f, up)
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    M = np.eye(4)
    M[0, :3], M[1, :3], M[2, :3] = s, u, -f
    M[:3, 3] = -M[:3, :3] @ eye
    return M


def _rotation(axis, angle):
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def _unit_vectors(seed, tag, n):
    u = uniform(seed, tag, 2 * n).reshape(n, 2)
    z = 2.0 * u[:, 0] - 1.0
    a = 2.0 * np.pi * u[:, 1]
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(a), r * np.sin(a), z], axis=1)


@dataclass
class ShaderParams:
    """Host-side vertex-shader inputs (all float32 except the integers)."""
    kind: int
    num_lights: int = 0
    iterations: int = 0
    spec_squarings: int = 5
    mvp: np.ndarray = None       # [16] row-major 4x4
    model: np.ndarray = None     # [12] row-major 3x4
    normal: np.ndarray = None    # [9]  row-major 3x3
    eye: np.ndarray = None       # [3]
    ambient: np.ndarray = None   # [3]
    kd: float = 0.8
    ks: float = 0.2
    katt: float = 0.05
    coef: np.ndarray = None      # [8] c0 c1 c2 c3 cvec.x cvec.y cvec.z 0
    lights: np.ndarray = None    # [16, 6] pos.xyz colour.rgb


def make_shader(kind: int, seed: int, num_lights: int = 0, iterations: int = 64,
                center=(0.0, 0.0, 0.0), radius: float = 1.0) -> ShaderParams:
    center = np.asarray(center, dtype=np.float64)
    d = _unit_vectors(seed, 21, 1)[0]
    axis = _unit_vectors(seed, 22, 1)[0]
    angle = float(uniform(seed, 23, 1)[0]) * 2.0 * np.pi
    R = _rotation(axis, angle)
    model = np.zeros((3, 4))
    model[:, :3] = R
    model[:, 3] = center - R @ center          # rotate about the mesh centre
    M4 = np.eye(4)
    M4[:3, :] = model
    eye = center + 2.5 * radius * d
    VP = _perspective(60.0, 16.0 / 9.0, 0.1, 100.0) @ _look_at(eye, center, np.array([0.0, 1.0, 0.0]))
    mvp = VP @ M4
    nmat = np.linalg.inv(R).T
    lights = np.zeros((MAX_LIGHTS, 6))
    if num_lights:
        lights[:num_lights, :3] = center + 3.0 * radius * _unit_vectors(seed, 24, num_lights)
        lights[:num_lights, 3:] = 0.2 + 0.8 * uniform(seed, 25, 3 * num_lights).reshape(num_lights, 3)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel().astype(np.float32))
    return ShaderParams(kind=kind, num_lights=num_lights, iterations=iterations, spec_squarings=5,
                        mvp=f32(mvp), model=f32(model), normal=f32(nmat), eye=f32(eye),
                        ambient=f32([0.05, 0.05, 0.05]), kd=0.8, ks=0.2, katt=0.05,
                        coef=f32([0.5, 0.5, -0.25, 0.125, 0.03, 0.02, 0.01, 0.0]),
                        lights=f32(lights).reshape(MAX_LIGHTS, 6))


def shader_for_mesh(mesh: Mesh, kind: int, seed: int, num_lights: int = 0,
                    iterations: int = 64) -> ShaderParams:
    p = mesh.vertices[:, :3].astype(np.float64)
    lo, hi = p.min(axis=0), p.max(axis=0)
    return make_shader(kind, seed, num_lights, iterations, center=(lo + hi) / 2,
                       radius=float(np.linalg.norm(hi - lo) / 2))


# --------------------------------------------------------------------------
# Named workloads (sizes as in the benchmark configurations)
# --------------------------------------------------------------------------
def grid64_scan_mvp(seed: int = 1):
    """64x64-vertex grid (4,096 vertices, 7,938 triangles), row-major order,
    MVP shader."""
    m = grid_mesh(64, 64, seed, "scan")
    return m, shader_for_mesh(m, SHADER_MVP, seed)


def icosphere8_hilbert_phong8(seed: int = 2, level: int = 8):
    """Icosphere subdivided 8 times (655,362 vertices, 1,310,720 triangles),
    Hilbert order with 5% local swaps in windows of 256, Phong with 8 lights."""
    m = icosphere_mesh(level, seed, "hilbert", swap_frac=0.05, swap_window=256)
    return m, shader_for_mesh(m, SHADER_PHONG, seed, num_lights=8)


def grid2048_offset64(order: str = "hilbert", seed: int = 4, n: int = 2048):
    """2048x2048-vertex grid (8,380,418 triangles) in Hilbert or fully random
    triangle order with the 64-iteration normal-offset shader."""
    m = grid_mesh(n, n, seed, order)
    return m, shader_for_mesh(m, SHADER_OFFSET, seed, iterations=64)


# --------------------------------------------------------------------------
# Serving workload: a pool of resident meshes and a Poisson request stream
# --------------------------------------------------------------------------
def serving_bases(seed: int = 11, grid_n: int = 1024, ico_level: int = 8):
    """Base meshes of the request pool: two grids of grid_n x grid_n vertices
    (about 2.09M triangles at 1024) and two icospheres (1.31M triangles at
    level 8), one of each in Hilbert and one in scan order."""
    return [grid_mesh(grid_n, grid_n, seed, "hilbert"), grid_mesh(grid_n, grid_n, seed + 1, "scan"),
            icosphere_mesh(ico_level, seed + 2, "hilbert"), icosphere_mesh(ico_level, seed + 3, "scan")]


def serving_pool(bases, seed: int = 12, n: int = 200, size_median: int = 20000, sigma: float = 1.5,
                 size_lo: int = 1000, size_hi: int = 2_000_000):
    """n meshes with sizes log-normal (median `size_median`, `sigma`) clamped
    to [size_lo, size_hi] and to the base: mesh m is a contiguous window
    (base m mod len(bases), first triangle, triangles) of a base index
    buffer, starting at a seeded triangle."""
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.exp(rng.normal(np.log(size_median), sigma, n)), size_lo, size_hi).astype(np.int64)
    pool = []
    for m in range(n):
        b = m % len(bases)
        T = bases[b].num_tris
        size = int(min(sizes[m], T))
        start = int(rng.integers(0, T - size + 1))
        pool.append((b, start, size))
    return pool


def serving_trace(pool, seed: int = 13, n: int = 2000, rate: float = 500.0, lights=(1, 16)):
    """Poisson arrivals at `rate` per second; a request draws a whole pool
    mesh, uniformly, with Phong lighting of a uniform number of lights."""
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1.0 / rate, n))
    arrival -= arrival[0]
    mesh = rng.integers(0, len(pool), n)
    size = np.array([pool[m][2] for m in mesh], dtype=np.int64)
    nl = rng.integers(lights[0], lights[1] + 1, n)
    return {"arrival": arrival, "size": size, "mesh": mesh, "lights": nl}


# --------------------------------------------------------------------------
# Random walk on a grid (Section 5, parallel random walk)
# --------------------------------------------------------------------------
class WalkSetup:
    """Inputs of the random-walk workload: an activity field over a G x G
    grid (float32, row-major, cell (x, y) at y * G + x), the move table
    (every offset within `radius`, scan order by dy then dx, with its
    step-length weight, float32) and the agents' packed cell keys
    (x | y << 16)."""

    def __init__(self, grid, activity, moves, weights, keys, seed):
        self.grid, self.activity, self.moves, self.weights, self.keys, self.seed = \
            grid, activity, moves, weights, keys, seed


def walk_setup(seed: int = 21, grid: int = 256, agents: int = 300_000, radius: int = 16,
               gaussians: int = 8, beta: float = 1.5, order: str = "hilbert") -> WalkSetup:
    """Activity = a floor of 1e-3 plus `gaussians` Gaussian bumps (centres
    uniform on the grid, sigma in [6, 24) cells, weight in [0.5, 1.5)),
    evaluated in float64 and stored as float32.  Moves: all (dx, dy) with
    1 <= dx^2 + dy^2 <= radius^2; the weight of a move of length d is
    d^-(1 + beta), a Levy-flight step-length law, rounded to float32.
    Agents start on uniformly drawn cells and are stored in the Hilbert
    order of those cells ("hilbert") or in the order drawn ("random")."""
    u = uniform(seed, 1, 4 * gaussians).reshape(gaussians, 4)
    cx, cy = u[:, 0] * grid, u[:, 1] * grid
    sig, w = 6.0 + 18.0 * u[:, 2], 0.5 + u[:, 3]
    y, x = np.mgrid[0:grid, 0:grid].astype(np.float64)
    act = np.full((grid, grid), 1e-3)
    for g in range(gaussians):
        act += w[g] * np.exp(-((x - cx[g]) ** 2 + (y - cy[g]) ** 2) / (2.0 * sig[g] ** 2))
    moves = [(dx, dy) for dy in range(-radius, radius + 1) for dx in range(-radius, radius + 1)
             if 1 <= dx * dx + dy * dy <= radius * radius]
    mv = np.array(moves, dtype=np.int8)
    d = np.sqrt((mv.astype(np.float64) ** 2).sum(1))
    weights = (d ** -(1.0 + beta)).astype(np.float32)
    r = u64_stream(seed, 2, 2 * agents)
    ax = (r[0::2] % np.uint64(grid)).astype(np.uint32)
    ay = (r[1::2] % np.uint64(grid)).astype(np.uint32)
    if order == "hilbert":   # agents stored in the Hilbert order of their starting cells
        bits = max(1, int(np.ceil(np.log2(grid))))
        perm = np.argsort(hilbert2d(ax.astype(np.uint64), ay.astype(np.uint64), bits), kind="stable")
        ax, ay = ax[perm], ay[perm]
    return WalkSetup(grid, act.astype(np.float32).ravel(), mv, weights, ax | (ay << np.uint32(16)), seed)


def walk_uniforms(seed: int, step: int, agents: int) -> np.ndarray:
    """Each agent's random number for one step: 24-bit uniforms in [0, 1),
    exact in float32."""
    return uniform(seed, 1000 + step, agents).astype(np.float32)
