"""Pins of the oracle's multi-level encoding (hierarchical encodings, Sec.
IV-A): a level small enough to be stored densely is the plain trilinear
interpolation (against scipy); the index of every vertex, read back by
probing vertex positions, has the published spatial-hash structure; and the
encoding feeds the renderer in place of the dense features."""
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _primes():
    vals = [int(l) for l in open(os.path.join(HERE, "golden", "hash_primes.txt")) if l.strip() and l[0] != "#"]
    assert len(vals) == 3
    return vals


def _model(res_levels, log2_size, tables, box=(0.0, 1.0)):
    dens = np.zeros((4, 4, 4), np.float32)
    return oracle.Model(dens, None, synth.make_mlp(1, in_dim=tables.shape[0] * tables.shape[2] + 27),
                        box_lo=(box[0],) * 3, box_hi=(box[1],) * 3,
                        hash_enc={"res": res_levels, "log2_size": log2_size, "tables": tables})


def test_dense_level_is_trilinear_interpolation():
    rng = np.random.default_rng(0)
    N, F, lg = 6, 3, 9        # (N+1)^3 = 343 <= 512: stored densely
    tab = rng.normal(0, 1, (1, 1 << lg, F)).astype(np.float32)
    m = _model((N,), lg, tab, box=(-1.0, 2.0))
    pos = rng.uniform(-1.0, 2.0, (500, 3)).astype(np.float32)
    got = oracle.encode(m, pos)
    grid = tab[0, :(N + 1) ** 3].reshape(N + 1, N + 1, N + 1, F).astype(np.float64)
    ax = np.linspace(-1.0, 2.0, N + 1)
    for f in range(F):
        want = RegularGridInterpolator((ax, ax, ax), grid[..., f])(pos.astype(np.float64))
        assert np.allclose(got[:, f], want, atol=1e-6)


def _probe(m, verts):
    """Table entry of each vertex: with table[e] = e and box [0, N], a
    position exactly on vertex v reads entry h(v) with weight 1."""
    return np.rint(oracle.encode(m, np.asarray(verts, np.float32))[:, 0]).astype(np.int64)


def test_hashed_level_index_structure():
    p1, p2, p3 = _primes()
    lg = 10
    T = 1 << lg
    N = 40                    # 41^3 > 1024: hashed
    tab = np.arange(T, dtype=np.float32).reshape(1, T, 1)
    m = _model((N,), lg, tab, box=(0.0, float(N)))
    # axis terms against the published constants
    e = _probe(m, [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 3, 0), (0, 0, 5)])
    assert list(e) == [0, p1 % T, p2 % T, p3 % T, (3 * p2) % (1 << 32) % T, (5 * p3) % (1 << 32) % T]
    # XOR structure: h(x, y, z) = (x ^ h(0, y, z)) mod T for x < T, and likewise per axis
    rng = np.random.default_rng(1)
    v = rng.integers(0, N, (200, 3))
    h = _probe(m, v)
    hx = _probe(m, np.c_[np.zeros(200), v[:, 1:]])
    hy = _probe(m, np.c_[np.zeros(200), v[:, 1], np.zeros(200)])
    hz = _probe(m, np.c_[np.zeros((200, 2)), v[:, 2]])
    assert np.array_equal(h, (v[:, 0] * p1) % T ^ hx)
    assert np.array_equal(hx, hy ^ hz)
    assert h.min() >= 0 and h.max() < T


def test_dense_and_hashed_indexing_switch_at_the_table_size():
    N = 7                     # (N+1)^3 = 512
    v = np.array([(1, 2, 3), (7, 0, 5), (4, 4, 4)])
    dense = _model((N,), 9, np.arange(512, dtype=np.float32).reshape(1, 512, 1), box=(0.0, 7.0))
    assert list(_probe(dense, v)) == [(x * 8 + y) * 8 + z for x, y, z in v]
    hashed = _model((N,), 8, np.arange(256, dtype=np.float32).reshape(1, 256, 1), box=(0.0, 7.0))
    p1, p2, p3 = _primes()
    assert list(_probe(hashed, v)) == [((x * p1) ^ (y * p2 % (1 << 32)) ^ (z * p3 % (1 << 32))) % 256 for x, y, z in v]


def test_interpolation_between_probed_vertices():
    """Inside a cell the encoding is the trilinear blend of the 8 entries the
    probe finds at the cell's corners (hashed level, random table)."""
    rng = np.random.default_rng(2)
    lg, N, F = 10, 40, 3
    T = 1 << lg
    vals = rng.normal(0, 1, (T, F)).astype(np.float32)
    idx_model = _model((N,), lg, np.arange(T, dtype=np.float32).reshape(1, T, 1), box=(0.0, float(N)))
    m = _model((N,), lg, vals.reshape(1, T, F), box=(0.0, float(N)))
    pos = rng.uniform(0, N - 1e-3, (300, 3)).astype(np.float32)
    got = oracle.encode(m, pos)
    base = np.floor(pos).astype(np.int64)
    frac = pos.astype(np.float64) - base
    want = np.zeros((300, F))
    for c in range(8):
        d = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        e = _probe(idx_model, base + d)
        w = np.prod(np.where(d == 1, frac, 1 - frac), axis=1)
        want += w[:, None] * vals[e].astype(np.float64)
    assert np.allclose(got, want, atol=1e-9)


def test_levels_concatenate_and_render_uses_them():
    """Features are the levels in order; a render with the encoding equals a
    render with a dense grid holding the same per-sample features (one dense
    level on the density grid's own vertices)."""
    rng = np.random.default_rng(3)
    R = 9                     # density grid of 9^3 vertices = 8 cells per axis
    dens, _ = synth.make_scene(R, seed=4)
    feats = rng.normal(0, 0.3, (R, R, R, 12)).astype(np.float32)
    lg = 10                   # 9^3 = 729 <= 1024: dense, on the same vertices
    tab = np.zeros((4, 1 << lg, 3), np.float32)
    for l in range(4):
        tab[l, :R ** 3] = feats[..., 3 * l:3 * l + 3].reshape(-1, 3)
    mlp = synth.make_mlp(5)
    sh = float(synth.DENSITY_SHIFT)
    dense = oracle.Model(dens, feats, mlp, density_shift=sh)
    hashed = oracle.Model(dens, None, mlp, density_shift=sh,
                          hash_enc={"res": (R - 1,) * 4, "log2_size": lg, "tables": tab})
    o, d = synth.random_rays(64, seed=6)
    op = oracle.opts(64)
    a = oracle.render_rays(dense, op, o, d)
    b = oracle.render_rays(hashed, op, o, d)
    for x, y in zip(a, b):
        assert np.allclose(x, y, atol=1e-12)
