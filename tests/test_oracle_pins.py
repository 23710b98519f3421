"""Pins of the CPU oracle against facts it does not compute itself.

Each test checks the oracle against a closed form, a value the paper
prints, a special case that reduces to a textbook routine, a brute-force
enumeration on tiny inputs, or an exact hand-derived shader case, so that a
plausible mistake (dropped term, wrong index, wrong cut rule, transposed
operand, a missing clamp) fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import vro
from paper_1805_08893_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL = range(8)
REUSE = [vro.STATIC_BALLOT, vro.STATIC_SORT, vro.STATIC_HASH, vro.DYN_SORT, vro.DYN_HASH,
         vro.DYN_PHASH, vro.DYN_BALLOT]
SORTS = (vro.STATIC_SORT, vro.DYN_SORT)
DYN = (vro.DYN_SORT, vro.DYN_HASH, vro.DYN_PHASH, vro.DYN_BALLOT)
BALLOT = (vro.STATIC_BALLOT, vro.DYN_BALLOT)


def _identity_shader(kind=W.SHADER_MVP):
    sp = W.make_shader(kind, 0)
    sp.mvp = np.eye(4, dtype=np.float32).ravel()
    sp.model = np.eye(3, 4, dtype=np.float32).ravel()
    sp.normal = np.eye(3, dtype=np.float32).ravel()
    return sp


def _vbuf(p, n=(0, 0, 1), uv=(0.25, 0.75)):
    return np.array([[*p, *n, *uv]], dtype=np.float32)


# ---------------------------------------------------------------- brute force
def brute_units(idx, begin, end, cap, tmax):
    """Units as maximal feasible prefixes, by enumeration with Python sets."""
    units, cur = [], begin
    while cur < end:
        best = cur + 1
        for e in range(cur + 1, end + 1):
            if e - cur <= tmax and len(set(idx[3 * cur:3 * e].tolist())) <= cap:
                best = e
        units.append(cur)
        cur = best
    return units


def brute_draw(idx, strategy, batch_tris, max_unique):
    """Expected units / local ids / invocation counts written from the
    definitions: static ranges, maximal dynamic prefixes, rounds of <= 64
    distinct, ascending ranks (numpy.unique) or dict insertion order."""
    T = len(idx) // 3
    if strategy == vro.NAIVE:
        batches = list(range(T))
    elif strategy in DYN:
        batches = brute_units(idx, 0, T, max_unique, batch_tris)
    else:
        batches = list(range(0, T, batch_tris))
    batches.append(T)
    units = []
    for b in range(len(batches) - 1):
        if strategy in BALLOT:
            units += brute_units(idx, batches[b], batches[b + 1], 64, 1 << 30)
        else:
            units.append(batches[b])
    units.append(T)
    local, inv = np.zeros(3 * T, np.int64), []
    for u in range(len(units) - 1):
        seg = idx[3 * units[u]:3 * units[u + 1]]
        if strategy == vro.NAIVE:
            ids = np.arange(len(seg))
        elif strategy in SORTS:
            uq = np.unique(seg)
            ids = np.searchsorted(uq, seg)
        else:
            order = {}
            for v in seg.tolist():
                order.setdefault(v, len(order))
            ids = np.array([order[v] for v in seg.tolist()])
        local[3 * units[u]:3 * units[u + 1]] = ids
        inv.append(int(ids.max()) + 1 if len(ids) else 0)
    return np.array(units), local, np.array(inv)


def _check_against_brute(idx, V, strategy, bt, nu):
    verts = np.tile(np.arange(V, dtype=np.float32)[:, None], (1, 8))
    sp = _identity_shader()
    rc, r = vro.process_draw(idx, verts, sp, strategy, bt, {"max_unique": nu},
                             corners=False, verts=False, tris=False)
    assert rc == vro.OK
    units, local, inv = brute_draw(idx, strategy, bt, nu)
    np.testing.assert_array_equal(r["unit_offsets"], units)
    np.testing.assert_array_equal(r["unit_invocations"], inv)
    np.testing.assert_array_equal(r["local_idx"], local)
    assert int(r["counters"][0]) == int(inv.sum())


def test_brute_force_exhaustive_two_triangles():
    """Every index buffer of 2 triangles over 4 vertices, several caps."""
    for combo in itertools.product(range(4), repeat=6):
        idx = np.array(combo, dtype=np.uint32)
        for strategy, bt, nu in ((vro.DYN_HASH, 2, 3), (vro.DYN_SORT, 2, 4), (vro.DYN_BALLOT, 1, 3),
                                 (vro.STATIC_SORT, 1, 0), (vro.STATIC_HASH, 2, 0),
                                 (vro.STATIC_BALLOT, 2, 0), (vro.NAIVE, 1, 0)):
            _check_against_brute(idx, 4, strategy, bt, nu)


def test_brute_force_random_small():
    rng = np.random.default_rng(5)
    for trial in range(300):
        T = int(rng.integers(1, 40))
        V = int(rng.integers(1, 24))
        idx = rng.integers(0, V, 3 * T).astype(np.uint32)
        strategy = int(rng.integers(0, 8))
        if strategy in DYN:
            bt = int(rng.integers(1, 20))
            nu = int(rng.integers(3, 12))
        else:
            bt = int(rng.integers(1, 30))
            nu = 0
        _check_against_brute(idx, V, strategy, bt, nu)


def test_brute_force_ballot_rounds_overflow():
    """Ballot rounds on all-distinct and mixed streams where 64 binds."""
    rng = np.random.default_rng(9)
    for V in (64, 100, 1000):
        idx = rng.integers(0, V, 3 * 200).astype(np.uint32)
        for bt in (21, 22, 64, 200):
            _check_against_brute(idx, V, vro.STATIC_BALLOT, bt, 0)
    idx = np.arange(3 * 100, dtype=np.uint32)
    _check_against_brute(idx, 300, vro.STATIC_BALLOT, 100, 0)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [2, 3, 64])
def test_grid_closed_form(n):
    m = W.grid_mesh(n, n, 1, "scan")
    assert m.num_tris == 2 * (n - 1) ** 2
    assert vro.count_unique(m.indices, m.num_verts) == n * n


@pytest.mark.parametrize("k", [0, 1, 3, 5])
def test_icosphere_closed_form(k):
    m = W.icosphere_mesh(k, 2, "hilbert")
    assert m.num_tris == 20 * 4 ** k
    assert vro.count_unique(m.indices, m.num_verts) == 10 * 4 ** k + 2


def _table1_ideal():
    rows = []
    with open(os.path.join(GOLDEN, "table1_closed_mesh_ideal_reuse.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(float(line.split()[-1]))
    return rows


def test_ideal_reuse_matches_table1_closed_meshes():
    """Ideal reuse of a closed sphere-like mesh rounds to Table 1's .833,
    and each vertex is referenced about six times (Figure 1 caption)."""
    m = W.icosphere_mesh(5, 2, "scan")
    U = vro.count_unique(m.indices, m.num_verts)
    ideal = 1.0 - U / len(m.indices)
    assert round(ideal, 3) in _table1_ideal()
    assert abs(len(m.indices) / U - 6.0) < 0.01
    # the whole-mesh unit reaches it: static sort with N_p >= T shades U times
    rc, r = vro.process_draw(m.indices[:3 * 256], m.vertices, _identity_shader(), vro.STATIC_SORT, 256,
                             corners=False, verts=False)
    assert int(r["counters"][0]) == vro.count_unique(m.indices[:3 * 256], m.num_verts)


# ---------------------------------------------------------------- special cases
def test_s1_naive_three_per_triangle():
    m = W.grid_mesh(9, 7, 3, "random")
    rc, r = vro.process_draw(m.indices, m.vertices, _identity_shader(), vro.NAIVE, 1)
    assert rc == vro.OK and int(r["counters"][0]) == 3 * m.num_tris
    np.testing.assert_array_equal(r["local_idx"], np.tile([0, 1, 2], m.num_tris))


def test_s2_one_static_batch_is_global_sorted_unique():
    m = W.grid_mesh(10, 10, 3, "hilbert")
    sp = W.shader_for_mesh(m, W.SHADER_PHONG, 3, num_lights=4)
    rc, r = vro.process_draw(m.indices, m.vertices, sp, vro.STATIC_SORT, 256)
    uq = np.unique(m.indices)
    assert int(r["counters"][0]) == len(uq)
    np.testing.assert_array_equal(r["local_idx"], np.searchsorted(uq, m.indices))
    np.testing.assert_array_equal(r["verts"], vro.shade(sp, m.vertices[uq]))


def test_s3_dynamic_with_large_budget_equals_static():
    m = W.icosphere_mesh(3, 4, "hilbert")
    for st_dyn, st_static in ((vro.DYN_HASH, vro.STATIC_HASH), (vro.DYN_SORT, vro.STATIC_SORT)):
        _, a = vro.process_draw(m.indices, m.vertices, _identity_shader(), st_dyn, 64,
                                {"max_unique": 192}, corners=False, verts=False)
        _, b = vro.process_draw(m.indices, m.vertices, _identity_shader(), st_static, 64,
                                corners=False, verts=False)
        for key in ("unit_offsets", "unit_invocations", "local_idx", "tris"):
            np.testing.assert_array_equal(a[key], b[key])


def test_s4_ballot_with_small_batches_equals_hash():
    m = W.icosphere_mesh(3, 4, "random")
    _, a = vro.process_draw(m.indices, m.vertices, _identity_shader(), vro.STATIC_BALLOT, 21,
                            corners=False, verts=False)
    _, b = vro.process_draw(m.indices, m.vertices, _identity_shader(), vro.STATIC_HASH, 21,
                            corners=False, verts=False)
    for key in ("unit_offsets", "unit_invocations", "local_idx", "tris"):
        np.testing.assert_array_equal(a[key], b[key])


def test_s5_min_budget_all_distinct():
    T = 50
    idx = np.arange(3 * T, dtype=np.uint32)
    verts = np.zeros((3 * T, 8), np.float32)
    rc, r = vro.process_draw(idx, verts, _identity_shader(), vro.DYN_HASH, 10, {"max_unique": 3},
                             corners=False, verts=False)
    assert int(r["counters"][0]) == 3 * T and int(r["counters"][1]) == T


def test_s7_all_equal_indices():
    idx = np.zeros(3 * 100, dtype=np.uint32)
    verts = np.zeros((1, 8), np.float32)
    for st, bt, nunits in ((vro.STATIC_SORT, 7, 15), (vro.STATIC_BALLOT, 7, 15), (vro.DYN_HASH, 33, 4),
                           (vro.DYN_BALLOT, 512, 1)):
        rc, r = vro.process_draw(idx, verts, _identity_shader(), st, bt, corners=False, verts=False)
        assert int(r["counters"][1]) == nunits and int(r["counters"][0]) == nunits


def test_empty_draw():
    rc, r = vro.process_draw(np.zeros(0, np.uint32), np.zeros((4, 8), np.float32), _identity_shader(),
                             vro.DYN_HASH, 64)
    assert rc == vro.OK and r["counters"].tolist() == [0, 0, 0, 0]


def test_index_out_of_range_is_reported():
    idx = np.array([0, 1, 4], dtype=np.uint32)
    rc, r = vro.process_draw(idx, np.zeros((4, 8), np.float32), _identity_shader(), vro.STATIC_SORT, 4)
    assert rc == vro.ERR_INDEX_RANGE and int(r["counters"][3]) == vro.ERR_INDEX_RANGE


def test_argument_errors():
    idx = np.zeros(6, np.uint32)
    v = np.zeros((1, 8), np.float32)
    sp = _identity_shader()
    assert vro.process_draw(idx[:5], v, sp, vro.NAIVE, 1)[0] == vro.ERR_ARG          # not triangles
    assert vro.process_draw(idx, v, sp, 9, 1)[0] == vro.ERR_ARG                      # strategy
    assert vro.process_draw(idx, v, sp, vro.STATIC_SORT, 0)[0] == vro.ERR_ARG        # batch 0
    assert vro.process_draw(idx, v, sp, vro.STATIC_SORT, 257)[0] == vro.ERR_ARG      # batch cap
    assert vro.process_draw(idx, v, sp, vro.DYN_HASH, 64, {"max_unique": 2})[0] == vro.ERR_ARG
    assert vro.process_draw(idx, v, sp, vro.DYN_HASH, 64, {"max_unique": 4097})[0] == vro.ERR_ARG
    assert vro.process_draw(idx, v, sp, vro.DYN_HASH, 64, {"hash_slots": 100})[0] == vro.ERR_ARG
    sp.num_lights = 17
    assert vro.process_draw(idx, v, sp, vro.NAIVE, 1)[0] == vro.ERR_ARG


def test_dynamic_units_satisfy_caps_and_are_maximal():
    m = W.icosphere_mesh(4, 6, "hilbert", swap_frac=0.05)
    for nu, tmax in ((64, 85), (256, 341), (128, 128), (7, 1000)):
        offs = vro.plan_dynamic(m.indices, m.num_verts, nu, tmax)
        for b in range(len(offs) - 1):
            t0, t1 = int(offs[b]), int(offs[b + 1])
            assert 0 < t1 - t0 <= tmax
            assert len(set(m.indices[3 * t0:3 * t1].tolist())) <= nu
            if t1 < m.num_tris and t1 - t0 < tmax:
                assert len(set(m.indices[3 * t0:3 * t1 + 3].tolist())) > nu


# ---------------------------------------------------------------- FIFO cache
def test_fifo_hand_examples():
    strip = np.array([0, 1, 2, 1, 2, 3, 2, 3, 4], np.uint32)
    assert vro.fifo_misses(strip, 5, 3) == 5
    # FIFO (unlike LRU) does not refresh on a hit: 0 1 0 2 0 3 with k=2
    seq = np.array([0, 1, 0, 2, 0, 3], np.uint32)
    assert vro.fifo_misses(seq, 4, 2) == 5
    m = W.icosphere_mesh(3, 1, "random")
    U = vro.count_unique(m.indices, m.num_verts)
    assert vro.fifo_misses(m.indices, m.num_verts, U) == U
    assert vro.fifo_misses(m.indices, m.num_verts, 0) == len(m.indices)


# ---------------------------------------------------------------- shading
def test_mvp_identity_and_affine_exact():
    sp = _identity_shader()
    out = vro.shade(sp, _vbuf((0.5, -1.25, 3.0), (0, 0, 1)))[0]
    np.testing.assert_array_equal(out[:9], [0.5, -1.25, 3.0, 1.0, 0, 0, 1, 0.25, 0.75])
    np.testing.assert_array_equal(out[9:], sp.ambient)
    # scale-and-translate rows: x' = 2x + 3, y' = y/2 - 1, z' = z, w = z (row 3 = (0,0,1,0))
    sp.mvp = np.array([2, 0, 0, 3, 0, 0.5, 0, -1, 0, 0, 1, 0, 0, 0, 1, 0], np.float32)
    out = vro.shade(sp, _vbuf((0.5, -1.25, 3.0)))[0]
    np.testing.assert_array_equal(out[:4], [4.0, -1.625, 3.0, 3.0])
    # normal matrix rows are applied as dot products with the input normal
    sp.normal = np.array([0, 1, 0, 0, 0, 1, 1, 0, 0], np.float32)     # cyclic permutation
    out = vro.shade(sp, _vbuf((0, 0, 0), (0.0, 3.0, 4.0)))[0]
    np.testing.assert_array_equal(out[4:7], np.float32([0.6, 0.8, 0.0]))


def test_phong_light_along_normal_exact():
    sp = _identity_shader(W.SHADER_PHONG)
    sp.num_lights, sp.kd, sp.ks, sp.katt = 1, 0.75, 0.25, 0.25
    sp.ambient = np.float32([0.25, 0.125, 0.0])
    sp.eye = np.float32([0, 0, 5])
    lights = np.zeros((16, 6), np.float32)
    lights[0] = [0, 0, 2, 1.0, 0.5, 2.0]        # d2 = 4 -> att = 1/(1+0.25*4) = 0.5
    sp.lights = lights
    out = vro.shade(sp, _vbuf((0, 0, 0)))[0]
    # diffuse 1, reflection = n, view = n -> specular 1; k = 0.5*(0.25+0.75)
    np.testing.assert_array_equal(out[9:], np.float32([0.25 + 0.5, 0.125 + 0.25, 1.0]))
    # light behind the surface: both clamps give zero, colour = ambient
    lights[0, 2] = -2.0
    sp.lights = lights
    out = vro.shade(sp, _vbuf((0, 0, 0)))[0]
    np.testing.assert_array_equal(out[9:], sp.ambient)
    # specular only, reflection at 90 degrees from the view: light along +x,
    # normal +z -> ndl = 0 -> diffuse 0, r = -l -> dot(r, v) = 0
    lights[0] = [2, 0, 0, 1, 1, 1]
    sp.lights = lights
    out = vro.shade(sp, _vbuf((0, 0, 0)))[0]
    np.testing.assert_array_equal(out[9:], sp.ambient)


def test_phong_specular_exponent():
    """Mirror geometry with cos = 1/2 between reflection and view: the
    specular term is (1/2)^(2^s) exactly."""
    sp = _identity_shader(W.SHADER_PHONG)
    sp.num_lights, sp.kd, sp.ks, sp.katt = 1, 0.0, 1.0, 0.0
    sp.ambient = np.float32([0, 0, 0])
    lights = np.zeros((16, 6), np.float32)
    lights[0] = [0, 0, 1, 1, 1, 1]              # light along the normal: r = n
    sp.lights = lights
    # view direction (sqrt(3)/2, 0, 1/2) is not exact in float32; instead put
    # the eye at (x, 0, 1) with |(x,0,1)| = 2 -> x = sqrt(3): check vs float64
    for s in (0, 1, 3, 5):
        sp.spec_squarings = s
        sp.eye = np.float32([math.sqrt(3.0), 0.0, 1.0])
        o32 = vro.shade(sp, _vbuf((0, 0, 0)))[0]
        expect = 0.5 ** (2 ** s)
        assert abs(o32[9] - expect) <= 1e-6 * max(expect, 1e-30) * (2 ** s) + 1e-12


# A model matrix that is neither symmetric nor an involution: a cyclic axis
# permutation plus a translation, all entries powers of two or zero, so the
# world position is exact.  Read column-major or transposed it gives another
# point.  w = (p.y + 1, p.z - 2, p.x + 1/2).
PERM_MODEL = np.array([0, 1, 0, 1.0,
                       0, 0, 1, -2.0,
                       1, 0, 0, 0.5], np.float32)


def _perm_world(p):
    return np.float32([p[1] + 1.0, p[2] - 2.0, p[0] + 0.5])


def phong_on_axis_shader(model, p, offsets, colours, katt, ambient, kd=0.75, ks=0.25):
    """Phong with lights at world offsets (0, 0, dz) above the vertex's world
    position w = model (p, 1), the normal +z and the eye at w + (0, 0, 5)."""
    sp = _identity_shader(W.SHADER_PHONG)
    sp.model = np.asarray(model, np.float32)
    sp.kd, sp.ks, sp.katt = kd, ks, katt
    sp.ambient = np.float32(ambient)
    sp.spec_squarings = 5
    w = _perm_world(p) if model is PERM_MODEL else np.float32(p)
    sp.eye = w + np.float32([0, 0, 5])
    lights = np.zeros((16, 6), np.float32)
    for l, (dz, c) in enumerate(zip(offsets, colours)):
        lights[l, :3] = w + np.float32([0, 0, dz])
        lights[l, 3:] = c
    sp.lights = lights
    sp.num_lights = len(offsets)
    return sp


def _phong_on_axis(model, p, *args, **kw):
    return vro.shade(phong_on_axis_shader(model, p, *args, **kw), _vbuf(p))[0]


# (p, light heights, colours, katt, ambient, expected rgb): the hand cases
# below, also run through the GPU path
ULP1 = 2.0 ** -23
PHONG_HAND_CASES = [
    ((0.5, -1.25, 3.0), [2.0], [(1.0, 0.5, 2.0)], 0.25, (0.25, 0.125, 0.0), (0.75, 0.375, 1.0)),
    ((0.5, -1.25, 3.0), [1.0, 3.0, 1.0], [(2.0, 0.0, 0.0), (0.0, 4.0, 0.0), (0.0, 0.0, 8.0)], 7.0,
     (0.0, 0.0, 0.0), (0.25, 0.0625, 1.0)),
    ((0.5, -1.25, 3.0), [1.0, 2.0], [(0.75 * ULP1, 0.5 * ULP1, 0.0), (0.5 * ULP1, 0.75 * ULP1, 0.0)], 0.0,
     (1.0, 1.0, 1.0), (1.0 + 2 * ULP1, 1.0 + ULP1, 1.0)),
]


def test_phong_world_position_uses_row_major_model():
    """The lighting sees the world position model (p, 1) with the 3x4 model
    matrix stored row-major.  With the light 2 above w along the normal and
    the eye above it, diffuse = specular = 1 and att = 1/(1 + 1/4 * 4) = 1/2,
    so the colour is ambient + (1/2) * light colour exactly; any other world
    position puts the light off the normal and changes it."""
    for p in ((0.5, -1.25, 3.0), (-2.0, 0.25, 0.5), (1.0, 2.0, -0.75)):
        out = _phong_on_axis(PERM_MODEL, p, [2.0], [(1.0, 0.5, 2.0)], 0.25, (0.25, 0.125, 0.0))
        np.testing.assert_array_equal(out[9:], np.float32([0.75, 0.375, 1.0]))
        # the model matrix feeds lighting only: clip = mvp (p, 1) = (p, 1)
        np.testing.assert_array_equal(out[:4], np.float32([*p, 1.0]))


def test_phong_each_light_with_its_own_position_colour_and_attenuation():
    """Three lights on the normal at heights 1, 3 and 1 with katt = 7:
    att = 1/(1 + 7) = 1/8, 1/(1 + 63) = 1/64 and 1/8 (powers of two), and
    diffuse = specular = 1 with kd + ks = 1, so light l adds att_l * colour_l
    exactly.  Colours are distinct powers of two per channel, so dropping or
    repeating a light, or pairing a position with another light's colour,
    changes the sum."""
    cols = [(2.0, 0.0, 0.0), (0.0, 4.0, 0.0), (0.0, 0.0, 8.0)]
    out = _phong_on_axis(PERM_MODEL, (0.5, -1.25, 3.0), [1.0, 3.0, 1.0], cols, 7.0, (0.0, 0.0, 0.0))
    np.testing.assert_array_equal(out[9:], np.float32([2.0 / 8, 4.0 / 64, 8.0 / 8]))
    # the first light alone, and the first two: the loop runs l = 0 .. L-1
    out = _phong_on_axis(PERM_MODEL, (0.5, -1.25, 3.0), [1.0], cols[:1], 7.0, (0.0, 0.0, 0.0))
    np.testing.assert_array_equal(out[9:], np.float32([0.25, 0.0, 0.0]))
    out = _phong_on_axis(PERM_MODEL, (0.5, -1.25, 3.0), [1.0, 3.0], cols[:2], 7.0, (0.0, 0.0, 0.0))
    np.testing.assert_array_equal(out[9:], np.float32([0.25, 0.0625, 0.0]))


def test_phong_lights_accumulate_in_order():
    """The colour is accumulated light 0 first, one rounded fma per light.
    With ambient 1, k = 1 per light (katt = 0, light on the normal) and
    contributions of 3/4 and 1/2 ulp(1): in order 0, 1 the x channel rounds
    1 + 3/4 ulp up to 1 + ulp, then 1 + 3/2 ulp ties to even 1 + 2 ulp; the
    y channel takes 1/2 ulp first (a tie, back to 1) and then 3/4 ulp, giving
    1 + ulp.  The reverse order swaps the two results."""
    ulp = 2.0 ** -23
    cols = [(0.75 * ulp, 0.5 * ulp, 0.0), (0.5 * ulp, 0.75 * ulp, 0.0)]
    out = _phong_on_axis(PERM_MODEL, (0.5, -1.25, 3.0), [1.0, 2.0], cols, 0.0, (1.0, 1.0, 1.0))
    np.testing.assert_array_equal(out[9:], np.float32([1.0 + 2 * ulp, 1.0 + ulp, 1.0]))
    out = _phong_on_axis(PERM_MODEL, (0.5, -1.25, 3.0), [2.0, 1.0], cols[::-1], 0.0, (1.0, 1.0, 1.0))
    np.testing.assert_array_equal(out[9:], np.float32([1.0 + ulp, 1.0 + 2 * ulp, 1.0]))


def test_offset_reaches_fixed_point():
    """64 relaxation steps converge to the real root of
    c3 h^3 + c2 h^2 + (c1 - 1) h + dot(cvec, p) = 0 (contraction ~0.75)."""
    sp = _identity_shader(W.SHADER_OFFSET)
    sp.iterations = 64
    c = sp.coef.astype(np.float64)
    for p in ((0.3, -0.2, 0.9), (1.0, 1.0, 1.0), (-2.0, 0.5, 0.1)):
        out = vro.shade(sp, _vbuf(p, (0, 0, 1)))[0]
        ph = float(np.dot(c[4:7], p))
        roots = np.roots([c[3], c[2], c[1] - 1.0, ph])
        real = roots[np.abs(roots.imag) < 1e-12].real
        h = real[np.argmin(np.abs(real))]
        assert abs(out[0] - np.float32(p[0])) == 0 and abs(out[1] - np.float32(p[1])) == 0
        assert abs(float(out[2]) - (p[2] + h)) < 4e-6
    sp.iterations = 0                            # no refinement: p unchanged
    out = vro.shade(sp, _vbuf((0.3, -0.2, 0.9)))[0]
    np.testing.assert_array_equal(out[:3], np.float32([0.3, -0.2, 0.9]))


@pytest.mark.parametrize("kind,lights", [(W.SHADER_MVP, 0), (W.SHADER_PHONG, 8), (W.SHADER_PHONG, 16),
                                         (W.SHADER_OFFSET, 0)])
def test_fp32_program_within_rounding_of_fp64(kind, lights):
    """The FP32 program stays within a derived bound of the same program in
    float64: a few units in the last place per output, scaled by the
    magnitudes involved (x32 for the specular power)."""
    m = W.icosphere_mesh(3, 8, "scan")
    sp = W.shader_for_mesh(m, kind, 8, num_lights=lights)
    o32 = vro.shade(sp, m.vertices).astype(np.float64)
    o64 = vro.shade(sp, m.vertices, f64=True)
    scale = np.maximum(1.0, np.abs(o64))
    rel = np.abs(o32 - o64) / scale
    assert rel.max() < 64 * 2.0 ** -23, rel.max()


def test_corners_equal_naive_shading_all_strategies():
    """Invariant: whatever the strategy, corner k is the shaded vertex
    idx[k] (bitwise), and all strategies emit identical corners."""
    m = W.icosphere_mesh(3, 3, "hilbert", swap_frac=0.05)
    sp = W.shader_for_mesh(m, W.SHADER_PHONG, 3, num_lights=4)
    ref = vro.shade(sp, m.vertices[m.indices])
    for st in ALL:
        rc, r = vro.process_draw(m.indices, m.vertices, sp, st, 64)
        np.testing.assert_array_equal(r["corners"], ref)
        np.testing.assert_array_equal(r["verts"][r["tris"]], ref)
        inv, U = int(r["counters"][0]), int(r["counters"][2])
        assert U <= inv <= len(m.indices)


def test_multi_two_pass_reference():
    """The two-pass reference (Section 4.2, Table 2): every vertex of the
    buffer is shaded once, referenced or not, and corners are gathered from
    the shaded buffer.  Pins: invocations are V (not U), the shaded list is
    the buffer in vertex order, the assembled indices are the input indices,
    one unit spans the draw, and the corners equal naive shading bitwise."""
    m = W.grid_mesh(9, 7, 5, "hilbert")
    rng = np.random.default_rng(3)
    extra = rng.random((13, 8), dtype=np.float32)                # 13 unreferenced vertices
    vb = np.concatenate([m.vertices, extra])
    sp = W.shader_for_mesh(m, W.SHADER_PHONG, 2, num_lights=3)
    rc, r = vro.process_draw(m.indices, vb, sp, vro.MULTI, 1)
    assert rc == vro.OK
    V, U, T = len(vb), len(np.unique(m.indices)), m.num_tris
    assert r["counters"].tolist() == [V, 1, U, 0]
    np.testing.assert_array_equal(r["verts"], vro.shade(sp, vb))
    np.testing.assert_array_equal(r["tris"], m.indices)
    assert r["unit_offsets"].tolist() == [0, T] and r["unit_invocations"].tolist() == [V]
    rc, nv = vro.process_draw(m.indices, vb, sp, vro.NAIVE, 1)
    np.testing.assert_array_equal(r["corners"], nv["corners"])
    # an empty draw shades nothing
    rc, e = vro.process_draw(np.zeros(0, np.uint32), vb, sp, vro.MULTI, 1)
    assert rc == vro.OK and e["counters"].tolist() == [0, 0, 0, 0]


def test_multi_argument_rules():
    """Local ids are not defined for the single buffer-sized unit, and the
    shaded list needs room for all V vertices, not 3T."""
    import ctypes as C
    idx = np.array([0, 1, 2], np.uint32)
    sh = vro.make_shader(_identity_shader())
    lid = np.zeros(3, np.uint16)
    verts = np.zeros((8, 12), np.float32)
    def check(local, vcap):
        out = vro.Outputs(None, None, verts.ctypes.data, vcap, lid.ctypes.data if local else None, None, None, 0,
                          None)
        return vro.lib().vro_check_args(3, 8, C.byref(sh), vro.MULTI, 1, None, C.byref(out), None)
    assert check(False, 8) == vro.OK
    assert check(True, 8) == vro.ERR_ARG
    assert check(False, 7) == vro.ERR_CAPACITY     # 3T = 3 would do for the batched strategies
    assert vro.units_bound(vro.MULTI, 1000, 1) == 1


def test_plan_of_a_prefix_is_the_cut_plan():
    """Greedy batching closes a batch without looking past it, so the plan of
    the first T' triangles equals the plan of the whole stream cut at T'
    (batches starting before T', the last one ending at T').  The request
    server relies on this to serve prefixes of resident meshes."""
    meshes = [W.grid_mesh(30, 20, 3, "hilbert"), W.icosphere_mesh(3, 4, "random"),
              W.grid_mesh(25, 25, 5, "scan")]
    rng = np.random.default_rng(9)
    for m in meshes:
        for nu, bt in ((9, 3), (64, 21), (256, 256), (341, 512)):
            full = vro.plan_dynamic(m.indices, m.num_verts, nu, bt)
            for Tp in list(rng.integers(1, m.num_tris, 12)) + [1, m.num_tris]:
                Tp = int(Tp)
                own = vro.plan_dynamic(m.indices[:3 * Tp], m.num_verts, nu, bt)
                starts = full[:-1]
                cut = np.concatenate([starts[starts < Tp], [Tp]]).astype(np.uint32)
                assert np.array_equal(own, cut), (m.name, nu, bt, Tp)


def test_plan_is_the_aligned_chain_when_every_window_fits():
    """If every aligned window of N_pmax triangles holds at most N_u distinct
    indices, greedy batching cuts exactly at multiples of N_pmax (every
    prefix of such a window also fits).  The device planner takes this as a
    fast path after checking the windows."""
    cases = 0
    for m in (W.grid_mesh(40, 30, 2, "hilbert"), W.icosphere_mesh(4, 3, "hilbert"), W.grid_mesh(50, 20, 4, "scan")):
        T = m.num_tris
        for nu, bt in ((256, 256), (64, 21), (100, 33), (512, 341), (40, 16)):
            fits = all(len(np.unique(m.indices[3 * t:3 * min(T, t + bt)])) <= nu for t in range(0, T, bt))
            plan = vro.plan_dynamic(m.indices, m.num_verts, nu, bt)
            aligned = np.concatenate([np.arange(0, T, bt), [T]]).astype(np.uint32)
            if fits:
                cases += 1
                assert np.array_equal(plan, aligned), (m.name, nu, bt)
    assert cases >= 8


# ------------------------------------------------ parallel caches (Table 1)
def _lru_hits(stream, cap):
    """Textbook sequential LRU cache of `cap` entries: hits."""
    from collections import OrderedDict
    c, hits = OrderedDict(), 0
    for v in stream:
        if v in c:
            hits += 1
            c.move_to_end(v)
        else:
            c[v] = True
            if len(c) > cap:
                c.popitem(last=False)
    return hits


def test_parallel_cache_one_processor_is_a_textbook_lru():
    rng = np.random.default_rng(11)
    for trial in range(20):
        V = int(rng.integers(2, 40))
        s = rng.integers(0, V, int(rng.integers(1, 300))).astype(np.uint32)
        for cap in (1, 2, 5, 17, 64):
            assert vro.parallel_cache_hits(s, V, 1, 1, cap) == _lru_hits(s.tolist(), cap), (trial, cap)
    # capacity at least the distinct count: every repeat hits (the ideal reuse)
    m = W.grid_mesh(12, 10, 2, "hilbert")
    U = len(np.unique(m.indices))
    assert vro.parallel_cache_hits(m.indices, m.num_verts, 1, 1, U) == len(m.indices) - U
    # more capacity never loses a hit (LRU inclusion)
    h = [vro.parallel_cache_hits(m.indices, m.num_verts, 1, 1, c) for c in (1, 4, 16, 64, 256)]
    assert h == sorted(h)


def test_parallel_cache_concurrency_and_assignment():
    s = np.array([0, 0, 0, 1, 1, 2], np.uint32)
    assert vro.parallel_cache_hits(s, 3, 1, 1, 8) == 3
    assert vro.parallel_cache_hits(s, 3, 1, 6, 8) == 0          # one cycle: every duplicate is concurrent
    assert vro.parallel_cache_hits(s, 3, 1, 3, 8) == 0          # cycles [0 0 0] [1 1 2]: nothing cached yet
    assert vro.parallel_cache_hits(np.array([5, 6, 5, 6], np.uint32), 7, 1, 2, 8) == 2
    m = W.grid_mesh(20, 16, 3, "hilbert")
    n, V, N = len(m.indices), m.num_verts, 48
    chunks = -(-n // N)
    # as many processors as chunks: no processor ever sees a second cycle
    for contiguous in (True, False):
        assert vro.parallel_cache_hits(m.indices, V, chunks, N, 64, contiguous) == 0
    # processors share nothing: the total is the sum over each processor's
    # own chunk sequence run on one processor
    P = 5
    run = -(-chunks // P)
    for contiguous in (True, False):
        tot = 0
        for p in range(P):
            ids = range(p * run, min(chunks, (p + 1) * run)) if contiguous else range(p, chunks, P)
            sub = np.concatenate([m.indices[c * N:(c + 1) * N] for c in ids]) if len(ids) else np.zeros(0, np.uint32)
            tot += vro.parallel_cache_hits(sub, V, 1, N, 64)
        assert vro.parallel_cache_hits(m.indices, V, P, N, 64, contiguous) == tot
    assert vro.parallel_cache_hits(np.array([0, 9], np.uint32), 5, 1, 1, 4) == -1   # index out of range


# ------------------------------------------------- random walk (Section 5)
def _small_walk(seed=5, grid=24, agents=3000, radius=5):
    return W.walk_setup(seed, grid=grid, agents=agents, radius=radius, gaussians=3)


def test_walk_options_are_the_top8_by_brute_force():
    """A cell's options equal a full sort of every in-grid move by
    (likelihood descending, move index ascending), likelihood being one FP32
    product, including corner and edge cells with few moves."""
    s = _small_walk()
    G, mv = s.grid, s.moves.astype(np.int64)
    A = s.activity.reshape(G, G)
    for (x, y) in [(0, 0), (G - 1, G - 1), (0, 11), (7, 13), (G - 1, 0), (12, 12)]:
        tx, ty = x + mv[:, 0], y + mv[:, 1]
        ok = (tx >= 0) & (ty >= 0) & (tx < G) & (ty < G)
        m = np.nonzero(ok)[0]
        l = A[ty[m], tx[m]] * s.weights[m]                    # float32 x float32
        order = np.lexsort((m, -l.astype(np.float64)))[:8]
        L, mi = vro.walk_options(x, y, s)
        np.testing.assert_array_equal(mi, m[order])
        np.testing.assert_array_equal(L.view(np.uint32), l[order].view(np.uint32))
    # a flat field: ties everywhere, so the 8 lowest-indexed moves of the
    # largest weight (the four unit steps, then the four diagonals) win
    flat = _small_walk()
    flat.activity = np.ones_like(flat.activity)
    L, mi = vro.walk_options(10, 10, flat)
    d2 = (flat.moves.astype(np.int64) ** 2).sum(1)
    assert sorted(d2[mi].tolist()) == [1, 1, 1, 1, 2, 2, 2, 2]
    assert mi[:4].tolist() == sorted(mi[:4].tolist())


def test_walk_choice_follows_the_running_sum():
    s = _small_walk()
    L, mi = vro.walk_options(9, 4, s)
    cum = np.cumsum(L, dtype=np.float32)                        # sequential FP32 sums
    key = 9 | (4 << 16)
    for u in (0.0, 1e-7, 0.25, 0.5, 0.75, 0.999999):
        t = np.float32(u) * cum[-1]
        j = int(np.argmax(cum > t)) if (cum > t).any() else len(L) - 1
        dx, dy = (int(v) for v in s.moves[mi[j]])
        assert vro.walk_choose(key, u, L, mi, s.moves) == (9 + dx) | ((4 + dy) << 16), u
    assert vro.walk_choose(key, 0.3, np.zeros(8, np.float32), mi, s.moves) == key      # nothing to weigh: stay


def test_walk_step_batching_changes_only_the_counts():
    """Every strategy moves every agent to the same cell; NAIVE evaluates one
    cell per agent, the batched ones one per distinct cell of each batch."""
    s = _small_walk()
    keys = s.keys
    for step in range(3):
        u = W.walk_uniforms(s.seed, step, len(keys))
        rc, ref, c = vro.walk_step(keys, s, u, vro.NAIVE)
        assert rc == vro.OK and c[:2].tolist() == [len(keys), len(keys)]
        for strat in (vro.STATIC_SORT, vro.STATIC_HASH):
            for b in (1, 7, 256, 512):
                rc, got, c = vro.walk_step(keys, s, u, strat, b)
                assert rc == vro.OK
                np.testing.assert_array_equal(got, ref)
                d = sum(len(np.unique(keys[i:i + b])) for i in range(0, len(keys), b))
                assert c[:2].tolist() == [d, -(-len(keys) // b)]
        # every move stays in the grid
        assert ((ref & 0xFFFF) < s.grid).all() and ((ref >> 16) < s.grid).all()
        keys = ref


def test_walk_argument_rules():
    s = _small_walk(agents=10)
    u = np.zeros(10, np.float32)
    bad = s.keys.copy()
    bad[3] = s.grid                                             # x out of range
    assert vro.walk_step(bad, s, u, vro.STATIC_HASH, 8)[0] == vro.ERR_INDEX_RANGE
    assert vro.walk_step(s.keys, s, u, vro.STATIC_HASH, 513)[0] == vro.ERR_ARG
    assert vro.walk_step(s.keys, s, u, vro.DYN_HASH, 64)[0] == vro.ERR_ARG
    rc, out, c = vro.walk_step(s.keys[:0], s, u[:0], vro.STATIC_HASH, 8)
    assert rc == vro.OK and c.tolist() == [0, 0, 0, 0]


# ------------------------------------- triangle setup (the queue's consumer)
def _corners(tris_clip):
    """[T][3][4] clip positions -> corner rows [3T, 12] (other columns 0)."""
    c = np.zeros((3 * len(tris_clip), 12), np.float32)
    c[:, :4] = np.asarray(tris_clip, np.float32).reshape(-1, 4)
    return c


def test_setup_hand_cases():
    ccw = [[-0.5, -0.5, 0, 1], [0.5, -0.5, 0, 1], [0.0, 0.5, 0, 1]]
    rec, vis = vro.setup(_corners([ccw]), 100, 100)
    assert vis == 1
    assert rec[0, :5].tolist() == [25.0, 25.0, 75.0, 75.0, 2500.0] and rec[0, 5:6].view(np.uint32)[0] == 1
    rec, vis = vro.setup(_corners([ccw[::-1]]), 100, 100)          # clockwise: back facing
    assert vis == 0 and rec[0, 4] == -2500.0 and rec[0, 5:6].view(np.uint32)[0] == 0
    behind = [ccw[0], ccw[1], [0.0, 0.5, 0, -1]]                  # a corner behind the eye
    rec, vis = vro.setup(_corners([behind]), 100, 100)
    assert vis == 0 and not rec.any()
    off = [[2.0, 2.0, 0, 1], [3.0, 2.0, 0, 1], [2.5, 3.0, 0, 1]]    # right of and above the viewport
    rec, vis = vro.setup(_corners([off]), 100, 100)
    assert vis == 0 and rec[0, 4] > 0 and rec[0, 0] >= rec[0, 2]
    half = [[-2.0, -0.5, 0, 1], [0.5, -0.5, 0, 1], [0.0, 0.5, 0, 1]]   # partly left of it: clamped
    rec, vis = vro.setup(_corners([half]), 100, 100)
    assert vis == 1 and rec[0, 0] == 0.0


def test_setup_invariants():
    rng = np.random.default_rng(4)
    tri = rng.uniform(-1.5, 1.5, (500, 3, 4)).astype(np.float32)
    tri[:, :, 3] = rng.uniform(0.5, 2.0, (500, 3)).astype(np.float32)
    rec, vis = vro.setup(_corners(tri), 640, 480)
    # scaling a corner's homogeneous coordinates by 2 divides exactly: same record
    rec2, vis2 = vro.setup(_corners(tri * np.float32(2.0)), 640, 480)
    assert vis2 == vis and np.array_equal(rec.view(np.uint32), rec2.view(np.uint32))
    # the area's sign agrees with a float64 cross product wherever it is not tiny
    p = tri[:, :, :2].astype(np.float64) / tri[:, :, 3:4]
    sx, sy = (p[:, :, 0] + 1) * 320, (p[:, :, 1] + 1) * 240
    a64 = (sx[:, 1] - sx[:, 0]) * (sy[:, 2] - sy[:, 0]) - (sx[:, 2] - sx[:, 0]) * (sy[:, 1] - sy[:, 0])
    big = np.abs(a64) > 1e-2
    assert (np.sign(rec[big, 4]) == np.sign(a64[big])).all()
    np.testing.assert_allclose(rec[big, 4], a64[big], rtol=1e-3, atol=1e-2)
    # visible = positive area and a non-empty clamped box
    flags = rec[:, 5].view(np.uint32)
    want = (rec[:, 4] > 0) & (rec[:, 0] < rec[:, 2]) & (rec[:, 1] < rec[:, 3])
    assert np.array_equal(flags == 1, want) and vis == int(want.sum())
