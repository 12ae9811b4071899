"""Selector input features: two probe residual features and six density
statistics (learned first-floor selection).

The paper's rule uses the probe features r50 and r100 (Sec. 3.4); its
connectivity diagnostic is binary support at density >= 0.5, reported but never
a policy input (Tab. solver-config).  The six density statistics are not defined
in the paper; readings:

* fraction at floor  = #(rho == 0) / n_e
* mean               = mean(rho)
* min nonzero        = min(rho | rho > 0), 0 if every voxel is at the floor
* contrast           = log10(E_max / E_min) over non-floor voxels at the probe floor
* connectivity proxy = fraction of the elements along the loaded edge
                       (ex = nx-1, ez = 0) that are 6-connected through
                       {rho >= 0.5} to an element on the clamped face (ex = 0)
* grid size          = log10(n_DOF)
Probe features enter as log10(r50), log10(r100).
"""
import numpy as np
import scipy.ndimage as ndi


def density_stats(rho, nx, ny, nz, p, rho0):
    rho = np.asarray(rho, dtype=float)
    n_e = rho.size
    frac_floor = float(np.count_nonzero(rho == 0.0)) / n_e
    mean = float(rho.mean())
    nz_vals = rho[rho > 0]
    min_nonzero = float(nz_vals.min()) if nz_vals.size else 0.0
    if nz_vals.size:
        E = rho0 + (1.0 - rho0) * nz_vals ** p
        contrast = float(np.log10(E.max() / E.min()))
    else:
        contrast = 0.0
    conn = connectivity_proxy(rho, nx, ny, nz)
    size = float(np.log10(3 * (nx + 1) * (ny + 1) * (nz + 1)))
    return [frac_floor, mean, min_nonzero, contrast, conn, size]


def connectivity_proxy(rho, nx, ny, nz, thresh=0.5):
    solid = (np.asarray(rho).reshape(nz, ny, nx) >= thresh)   # [ez][ey][ex]
    labels, _ = ndi.label(solid)          # default structure = 6-connectivity
    clamp_labels = set(np.unique(labels[:, :, 0])) - {0}
    edge = labels[0, :, nx - 1]           # ez = 0, ex = nx-1, all ey
    hits = sum(1 for l in edge if l != 0 and l in clamp_labels)
    return hits / float(ny)


def selector_features(r50, r100, stats, floor=1e-300):
    return [float(np.log10(max(r50, floor))), float(np.log10(max(r100, floor)))] + list(stats)
