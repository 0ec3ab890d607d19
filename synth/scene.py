"""Synthetic dense-grid scenes and MLP weights.

Scene recipe (stand-in for a trained DirectVoxGO-style dense grid):

* raw density at each vertex = sum of 8 isotropic Gaussian blobs, centres
  uniform in [-1,1]^3, widths s uniform in [0.1,0.4], peaks lognormal
  (mu=3, sigma=0.5); the renderer applies softplus(raw + DENSITY_SHIFT) after
  interpolation;
* features: N(0,1) per vertex and channel, smoothed by the mean over the
  in-bounds part of the 3x3x3 window;
* vertices sit on the corners of the box [-1.5,1.5]^3 ("align corners").

Everything is generated in float64 and stored as float32; the FP16 copies
used by the precision path are the round-to-nearest-even of those float32
values (numpy's astype).
"""
import numpy as np

BOX_LO = (-1.5, -1.5, -1.5)
BOX_HI = (1.5, 1.5, 1.5)
N_FEAT = 12
# Additive shift applied before softplus, chosen so that empty space has
# density softplus(0 + shift) = 1e-3 (ten times below the occupancy cut).
DENSITY_SHIFT = float(np.float32(np.log(np.expm1(1e-3))))
# Occupancy cut on density used for empty-space skipping.
OCC_SIGMA = 1e-2


def _box_filter_inbounds(a):
    """Mean over the in-bounds part of the 3x3x3 window, per channel."""
    out = a
    for ax in range(3):
        n = out.shape[ax]
        s = out.copy()
        sl_lo = [slice(None)] * out.ndim
        sl_hi = [slice(None)] * out.ndim
        # s[i] += out[i-1] ; s[i] += out[i+1]
        sl_lo[ax] = slice(1, n)
        sl_hi[ax] = slice(0, n - 1)
        s[tuple(sl_lo)] += out[tuple(sl_hi)]
        s[tuple(sl_hi)] += out[tuple(sl_lo)]
        cnt = np.full(n, 3.0)
        cnt[0] = 2.0
        cnt[-1] = 2.0
        if n == 1:
            cnt[0] = 1.0
        shape = [1] * out.ndim
        shape[ax] = n
        out = s / cnt.reshape(shape)
    return out


def make_scene(res, seed=0, n_blobs=8, n_feat=N_FEAT):
    """Return (density_raw float32 [R,R,R], features float32 [R,R,R,C]).

    Index order is x slowest, z fastest; channel fastest for features.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, size=(n_blobs, 3))
    widths = rng.uniform(0.1, 0.4, size=n_blobs)
    peaks = np.exp(3.0 + 0.5 * rng.standard_normal(n_blobs))
    coords = np.linspace(BOX_LO[0], BOX_HI[0], res)
    X, Y, Z = np.meshgrid(coords, coords, coords, indexing="ij")
    raw = np.zeros((res, res, res), dtype=np.float64)
    for c, s, p in zip(centres, widths, peaks):
        d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        raw += p * np.exp(-d2 / (2.0 * s * s))
    del X, Y, Z
    feats = rng.standard_normal((res, res, res, n_feat))
    feats = _box_filter_inbounds(feats)
    return (np.ascontiguousarray(raw.astype(np.float32)),
            np.ascontiguousarray(feats.astype(np.float32)))


def make_model_grid(res, seed, n_feat=N_FEAT, std=0.01):
    """Trainable-model initial grids: N(0, std) raw density and features."""
    rng = np.random.default_rng(seed)
    dens = rng.normal(0.0, std, size=(res, res, res))
    feats = rng.normal(0.0, std, size=(res, res, res, n_feat))
    return (np.ascontiguousarray(dens.astype(np.float32)),
            np.ascontiguousarray(feats.astype(np.float32)))


def make_mlp(seed=1, in_dim=N_FEAT + 27, hidden=128, out_dim=3, bias_std=0.0):
    """Xavier-uniform weights drawn W0, W1, W2 in that order; row-major
    [out][in] float32.  Biases are zero unless bias_std > 0 (then drawn after
    the weights as N(0, bias_std), b0, b1, b2)."""
    rng = np.random.default_rng(seed)
    dims = [(hidden, in_dim), (hidden, hidden), (out_dim, hidden)]
    ws = []
    for fo, fi in dims:
        bound = np.sqrt(6.0 / (fi + fo))
        ws.append(rng.uniform(-bound, bound, size=(fo, fi)).astype(np.float32))
    bs = []
    for fo, _ in dims:
        if bias_std > 0:
            bs.append(rng.normal(0.0, bias_std, size=fo).astype(np.float32))
        else:
            bs.append(np.zeros(fo, dtype=np.float32))
    return {"w0": ws[0], "b0": bs[0], "w1": ws[1], "b1": bs[1],
            "w2": ws[2], "b2": bs[2]}


# multi-level (hash-grid) encoding: 4 levels x 3 features = the 12 MLP inputs
HASH_RES = (32, 64, 128, 256)
HASH_LOG2_SIZE = 19
HASH_FEAT = 3


def make_hash_tables(seed=30, res=HASH_RES, log2_size=HASH_LOG2_SIZE, feat=HASH_FEAT, std=0.2):
    """Feature tables [L][2^log2_size][F] of a multi-level encoding, entries
    drawn N(0, std) in float64 and stored float32 (every entry drawn, also
    the ones a dense level leaves unused)."""
    rng = np.random.default_rng(seed)
    t = rng.normal(0.0, std, (len(res), 1 << log2_size, feat))
    return {"res": tuple(int(r) for r in res), "log2_size": int(log2_size), "tables": t.astype(np.float32)}
