"""Seeded synthetic inputs: reproducibility and the structure each workload asks for."""
import hashlib

import numpy as np

from paper_2607_26382_amd import synth


def test_reproducible():
    a = synth.blobs(32, 16, 16, 1000)
    b = synth.blobs(32, 16, 16, 1000)
    assert hashlib.sha256(a.tobytes()).hexdigest() == hashlib.sha256(b.tobytes()).hexdigest()
    assert not np.array_equal(a, synth.blobs(32, 16, 16, 1001))


def test_blob_structure():
    rho = synth.blobs(64, 32, 32, 1000).reshape(32, 32, 64)
    blocks = rho.reshape(8, 4, 8, 4, 16, 4).transpose(0, 2, 4, 1, 3, 5).reshape(1024, 64)
    assert np.all(blocks.max(axis=1) == blocks.min(axis=1))      # constant per blob
    assert np.count_nonzero(blocks[:, 0] == 0) == 512             # exactly 50% of 1024 blobs at the floor
    nz = blocks[blocks[:, 0] > 0, 0]
    assert nz.min() >= 0.01 and nz.max() <= 1.0


def test_uniform_and_struts_ranges():
    u = synth.uniform(16, 8, 8, 0)
    assert u.shape == (1024,) and u.min() >= 0 and u.max() < 1
    s = synth.struts(32, 16, 16, 3000)
    assert s.min() >= 1e-3 and s.max() <= 1.0 and s.max() > 0.5


def test_bernoulli_binary():
    b = synth.bernoulli(10, 5, 5, 7, 0.3)
    assert set(np.unique(b)) <= {0.0, 1.0}


def test_selector_mixture():
    kinds = set()
    for seed in range(5_000_000, 5_000_040):
        dims, rho, kind = synth.selector_state(seed)
        assert dims in synth.SELECTOR_GRIDS and rho.size == dims[0] * dims[1] * dims[2]
        assert rho.min() >= 0.0 and rho.max() <= 1.0
        kinds.add(kind)
        d2, r2, k2 = synth.selector_state(seed)
        assert d2 == dims and k2 == kind and np.array_equal(r2, rho)
    assert kinds == {"blobs", "struts"}
    dims, rho, _ = synth.selector_state(6_000_000, dims=(64, 32, 32))
    assert dims == (64, 32, 32) and rho.size == 65536
