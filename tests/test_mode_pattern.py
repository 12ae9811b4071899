"""The mode-basis sparsity tables compiled into the library, checked against
Galerkin element matrices built here from their definition (CPU only).

Coarse element matrices of the 2:1 trilinear hierarchy are the element-wise
Galerkin products K_{l+1} = sum_c P_c^T K_l(child c) P_c (Tab. solver-config:
Galerkin coarse operators), with P_c the trilinear interpolation of a coarse
element's 24 DOFs to child c.  In the per-component Walsh basis of the node
index they have one fixed symmetric pattern at every level; the library stores
level >= 2 element matrices as the upper triangle of that pattern, so the
table must contain every nonzero the products produce.
"""
import itertools
import os
import re

import numpy as np

from oracle import ke as oke

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2607_26382_amd", "csrc", "tg_galerkin1_pattern.h")


def _header():
    txt = open(HDR).read()
    g1 = [tuple(map(int, m)) for m in re.findall(r"\{(\d+), (\d+), (\d+), (\d+)\}", txt)]
    nu = int(re.search(r"#define TG_GM_NU (\d+)", txt).group(1))
    body = txt[txt.index("kGMPairs"):]
    pairs = [tuple(map(int, m)) for m in re.findall(r"\{(\d+), (\d+)\}", body)]
    assert len(pairs) == nu
    return g1, pairs


def _child_interp(c):
    """24x24 trilinear interpolation from a parent element's nodal DOFs
    (3 a + comp, a = i + 2 j + 4 k) to those of child c (octant bits)."""
    P = np.zeros((24, 24))
    off = [(c >> b) & 1 for b in range(3)]
    for a in range(8):                     # child node, parent coordinates in [0, 1]
        x = [0.5 * (off[b] + ((a >> b) & 1)) for b in range(3)]
        for A in range(8):                 # parent node shape function
            w = np.prod([x[b] if (A >> b) & 1 else 1.0 - x[b] for b in range(3)])
            for comp in range(3):
                P[3 * a + comp, 3 * A + comp] = w
    return P


def _walsh():
    H8 = np.array([[np.prod([(2 * ((a >> b) & 1) - 1) if (m >> b) & 1 else 1 for b in range(3)])
                    for a in range(8)] for m in range(8)], float)
    return np.kron(H8, np.eye(3))


def _coarse(children):
    return sum(_child_interp(c).T @ children[c] @ _child_interp(c) for c in range(8))


def test_child_interpolation_reproduces_linear_fields():
    # P_c maps the nodal values of a linear displacement field to its values at
    # the child's nodes: a pin of the interpolation used below
    rng = np.random.default_rng(0)
    A, t = rng.standard_normal((3, 3)), rng.standard_normal(3)
    corner = lambda a, s, o: [s * (o[b] + ((a >> b) & 1)) for b in range(3)]
    u = np.concatenate([A @ np.array(corner(a, 1.0, (0, 0, 0))) + t for a in range(8)])
    for c in range(8):
        o = [(c >> b) & 1 for b in range(3)]
        uc = np.concatenate([A @ np.array(corner(a, 0.5, o)) + t for a in range(8)])
        assert np.allclose(_child_interp(c) @ u, uc)


def test_galerkin_levels_stay_on_the_stored_pattern():
    g1, pairs = _header()
    Ke = oke.ke()
    T = _walsh()
    rng = np.random.default_rng(7)
    sym = set(pairs) | {(c, r) for r, c in pairs}
    assert len(sym) == len({(r, c) for _, r, c, _ in g1}) == 279
    assert all(r <= c for r, c in pairs) and len(set(pairs)) == len(pairs)
    level1 = lambda: _coarse([rng.uniform(1e-3, 1.0) * Ke for _ in range(8)])
    mats = {1: level1()}
    mats[2] = _coarse([level1() for _ in range(8)])
    mats[3] = _coarse([_coarse([level1() for _ in range(8)]) for _ in range(8)])
    for lev, K in mats.items():
        Kh = T @ K @ T.T / 64.0
        scale = np.abs(Kh).max()
        nz = {(r, c) for r, c in itertools.product(range(24), range(24)) if abs(Kh[r, c]) > 1e-12 * scale}
        # every nonzero is stored, and with random moduli every stored entry is used
        assert nz == sym, f"level {lev}"
        # the nodal matrix is recovered from the stored entries alone
        # (T T^T = 8 I per component, so K = T^T Kh T)
        Ks = np.zeros((24, 24))
        for r, c in pairs:
            Ks[r, c] = Ks[c, r] = Kh[r, c]
        assert np.abs(T.T @ Ks @ T - K).max() <= 1e-12 * np.abs(K).max()
