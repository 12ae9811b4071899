"""Seeded synthetic density fields (inputs only; no solver arithmetic).

Both the HIP path and the CPU oracle are fed from these generators, which is the
only code the two sides share.  Every field is a flat float64 array of n_e
stored densities in [0, 1], x fastest ([nz][ny][nx]); a voxel "at the floor" is
stored as exactly 0.  All draws use numpy ``default_rng(seed)`` (PCG64), as the
paper does for its random states (Sec. 3.1, "Benchmark geometries").

Families (their shapes follow the workloads they stand in for):

* ``uniform``   - i.i.d. U[0,1) per voxel (the small plain-method cantilever).
* ``blobs``     - the grid is cut into blob^3-voxel blobs; a seeded permutation
                  puts exactly round(floor_frac * n_blobs) blobs at the floor and
                  gives every other blob one value ~ U[lo, hi] (severe states).
* ``struts``    - smoothly varying optimized-like field: background + sum of
                  Gaussian tubes around seeded segments, clipped at 1.
* ``bernoulli`` - the paper's binary stress fields: u ~ U(0,1)^n_e, solid
                  (1) where u < q, floor (0) elsewhere.
* ``selector_state`` - the mixture the learned first-floor selector is trained
                  and evaluated on: blob fields with a random floor fraction and
                  blob edge, or strut fields on an exact-floor background.
"""
import numpy as np


def uniform(nx, ny, nz, seed):
    return np.random.default_rng(seed).random(nx * ny * nz)


def blobs(nx, ny, nz, seed, blob=4, floor_frac=0.5, lo=0.01, hi=1.0, per_voxel=False):
    if nx % blob or ny % blob or nz % blob:
        raise ValueError("grid must be a multiple of the blob edge")
    bx, by, bz = nx // blob, ny // blob, nz // blob
    nb = bx * by * bz
    rng = np.random.default_rng(seed)
    n_floor = int(round(floor_frac * nb))
    perm = rng.permutation(nb)
    is_floor = np.zeros(nb, dtype=bool)
    is_floor[perm[:n_floor]] = True
    vals = rng.uniform(lo, hi, size=nb)
    vals[is_floor] = 0.0
    field = vals.reshape(bz, by, bx)
    field = np.repeat(np.repeat(np.repeat(field, blob, 0), blob, 1), blob, 2)
    if per_voxel:
        vox = rng.uniform(lo, hi, size=field.shape)
        field = np.where(field > 0, vox, 0.0)
    return np.ascontiguousarray(field).ravel()


def struts(nx, ny, nz, seed, n_struts=8, background=1e-3, sigma=(2.0, 6.0)):
    """Background plus Gaussian tubes (width sigma ~ U[sigma]) around seeded
    segments, clipped at 1."""
    rng = np.random.default_rng(seed)
    A = rng.uniform([0, 0, 0], [nx, ny, nz], size=(n_struts, 3))
    B = rng.uniform([0, 0, 0], [nx, ny, nz], size=(n_struts, 3))
    sig = rng.uniform(sigma[0], sigma[1], size=n_struts)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5,
                          np.arange(nx) + 0.5, indexing="ij")
    out = np.full((nz, ny, nx), background)
    for s in range(n_struts):
        d = B[s] - A[s]
        L2 = float(d @ d) or 1.0
        for zz in range(nz):          # slab at a time keeps memory bounded
            px, py, pz = x[zz] - A[s, 0], y[zz] - A[s, 1], z[zz] - A[s, 2]
            t = np.clip((px * d[0] + py * d[1] + pz * d[2]) / L2, 0.0, 1.0)
            qx, qy, qz = px - t * d[0], py - t * d[1], pz - t * d[2]
            out[zz] += np.exp(-(qx * qx + qy * qy + qz * qz) / (2 * sig[s] ** 2))
    return np.minimum(out, 1.0).ravel()


def bernoulli(nx, ny, nz, seed, q):
    u = np.random.default_rng(seed).random(nx * ny * nz)
    return np.where(u < q, 1.0, 0.0)


# Named workloads (grid, generator, seeds).
def plain_small(seed=0):
    """16x8x8 cantilever, i.i.d. uniform densities."""
    return (16, 8, 8), uniform(16, 8, 8, seed)


def severe(seed, nx=64, ny=32, nz=32):
    """Severe random state: 50% of 4^3 blobs at the floor, others U[0.01, 1]."""
    return (nx, ny, nz), blobs(nx, ny, nz, seed, 4, 0.5, 0.01, 1.0)


def strut_field(seed, nx=256, ny=128, nz=128):
    """Optimized-like smooth field: 8 seeded Gaussian struts on a 1e-3 floor."""
    return (nx, ny, nz), struts(nx, ny, nz, seed)


SELECTOR_GRIDS = ((32, 16, 16), (48, 24, 24), (64, 32, 32))


def selector_state(seed, dims=None):
    """One state of the selector's training / held-out mixture.

    The grid is drawn from SELECTOR_GRIDS unless given.  With probability 3/4
    a blob field: floor fraction q ~ U[0.3, 0.7], blob edge in {2, 4, 8},
    blob values U[0.01, 1]; otherwise a strut field with 4-12 struts of width
    sigma ~ U[0.05, 0.12] * ny on a zero background, where voxels below 1e-3
    are set to the floor (0).  Returns (dims, rho, kind)."""
    rng = np.random.default_rng(seed)
    if dims is None:
        dims = SELECTOR_GRIDS[int(rng.integers(len(SELECTOR_GRIDS)))]
    sub = int(rng.integers(2 ** 31))
    if rng.random() < 0.75:
        q = float(rng.uniform(0.3, 0.7))
        edge = (2, 4, 8)[int(rng.integers(3))]
        return dims, blobs(*dims, sub, blob=edge, floor_frac=q), "blobs"
    n = int(rng.integers(4, 13))
    ny = dims[1]
    rho = struts(*dims, sub, n_struts=n, background=0.0, sigma=(0.05 * ny, 0.12 * ny))
    return dims, np.where(rho < 1e-3, 0.0, rho), "struts"
