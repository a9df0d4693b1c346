"""Seeded synthetic problem inputs shared by the oracle and the HIP path.

This module builds *inputs only*: grid sizes, density fields, clamp masks and
nodal load vectors.  It holds none of the buckling method's arithmetic
(no element matrices, operators, solvers or eigen computations), so both the
CPU oracle and the GPU path may import it without sharing method code.

Conventions (used by every array produced here):
  * fine grid of ``nel = (nx, ny)`` or ``(nx, ny, nz)`` unit elements;
  * node index ``node = i + (nx+1)*(j + (ny+1)*k)`` (x fastest);
  * interleaved DOFs ``dof = d*node + c`` with ``d`` = dimension;
  * element index ``e = i + nx*(j + ny*k)``;
  * densities are float64 in ``[RHO_MIN, 1]``.

The density recipes mimic the paper's regimes (Sec. 3 and Sec. 5: stiffness
contrast E1/E0 = 1e6, grey-to-solid fields, solid regions at supports and
loads) on seeded Gaussian-filtered noise, since the paper's own designs and
geometries are not available.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

RHO_MIN = 1e-6


def n_nodes(nel):
    n = 1
    for v in nel:
        n *= v + 1
    return n


def n_dofs(nel):
    return len(nel) * n_nodes(nel)


def n_elems(nel):
    m = 1
    for v in nel:
        m *= v
    return m


def _smooth(field, sigma):
    return ndimage.gaussian_filter(field, sigma=sigma, mode="reflect", truncate=3.0)


def density_uniform_noise(nel, seed, mean=0.5, amp=0.1, sigma=2.0):
    """``mean + U(-amp, amp)`` i.i.d., Gaussian-smoothed, clipped to [RHO_MIN, 1].

    Shape of the returned array: flat ``m`` in element order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(reversed(nel))
    x = mean + rng.uniform(-amp, amp, size=shape)
    x = _smooth(x, sigma)
    return np.clip(x, RHO_MIN, 1.0).ravel().astype(np.float64)


def density_volume_fraction(nel, seed, volfrac, sigma, amp=0.35, solid_layers=2):
    """Gaussian-filtered standard normal field mapped to a target mean density.

    ``x = clip(volfrac + amp*g + c, RHO_MIN, 1)`` where ``g`` is the filtered
    noise standardised to zero mean / unit variance, the layers of elements at
    the clamped face (x = 0) and the loaded face (x = nx) are set solid, and
    the shift ``c`` is found by bisection so that ``mean(x) == volfrac``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(reversed(nel))
    g = _smooth(rng.standard_normal(size=shape), sigma)
    g = (g - g.mean()) / max(g.std(), 1e-300)
    band = np.zeros(shape, dtype=bool)
    if solid_layers > 0:
        band[..., :solid_layers] = True
        band[..., -solid_layers:] = True

    def field(c):
        x = np.clip(volfrac + amp * g + c, RHO_MIN, 1.0)
        x[band] = 1.0
        return x

    lo, hi = -2.0, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if field(mid).mean() > volfrac:
            hi = mid
        else:
            lo = mid
        if hi - lo < 1e-15:
            break
    return field(0.5 * (lo + hi)).ravel().astype(np.float64)


def clamp_mask(nel):
    """uint8 mask over all DOFs: 1 for every DOF of the nodes on the x = 0 face."""
    dim = len(nel)
    nn = [v + 1 for v in nel]
    idx = np.arange(n_nodes(nel)).reshape(tuple(reversed(nn)))
    nodes = idx[..., 0].ravel()
    mask = np.zeros(n_dofs(nel), dtype=np.uint8)
    for c in range(dim):
        mask[dim * nodes + c] = 1
    return mask


def _face_weights(nel):
    """Consistent nodal weights of a uniform unit traction on the x = nx face.

    Bilinear/linear shape functions integrate a uniform traction to nodal
    shares 1/4 (corner), 1/2 (edge), 1 (interior) in 3D, 1/2 (end) and 1
    (interior) in 2D, before normalisation to total 1.
    Returns (node indices, weights) with weights summing to 1.
    """
    dim = len(nel)
    nx = nel[0]
    if dim == 2:
        ny = nel[1]
        j = np.arange(ny + 1)
        w = np.ones(ny + 1)
        w[0] = w[-1] = 0.5
        nodes = nx + (nx + 1) * j
    else:
        ny, nz = nel[1], nel[2]
        jj, kk = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="xy")
        wy = np.ones(ny + 1)
        wy[0] = wy[-1] = 0.5
        wz = np.ones(nz + 1)
        wz[0] = wz[-1] = 0.5
        w = (wz[:, None] * wy[None, :]).ravel()
        nodes = (nx + (nx + 1) * (jj + (ny + 1) * kk)).ravel()
    return nodes, w / w.sum()


def axial_load(nel, magnitude=1.0):
    """Uniform compressive traction (-x direction) on the x = nx face, total ``magnitude``."""
    dim = len(nel)
    f = np.zeros(n_dofs(nel))
    nodes, w = _face_weights(nel)
    f[dim * nodes + 0] = -magnitude * w
    return f


def shear_load(nel, comp, magnitude=1.0):
    """Uniform traction along axis ``comp`` (1 = y, 2 = z) on the x = nx face."""
    dim = len(nel)
    f = np.zeros(n_dofs(nel))
    nodes, w = _face_weights(nel)
    f[dim * nodes + comp] = magnitude * w
    return f


def torsion_load(nel, moment=1.0):
    """Tangential nodal forces on the x = nx face, proportional to
    ``(0, -(z - zc), y - yc)`` and scaled to a unit twisting moment about x."""
    assert len(nel) == 3
    nx, ny, nz = nel
    nodes, w = _face_weights(nel)
    j = (nodes // (nx + 1)) % (ny + 1)
    k = nodes // ((nx + 1) * (ny + 1))
    dy = j - ny / 2.0
    dz = k - nz / 2.0
    fy = -dz * w
    fz = dy * w
    mom = np.sum(dy * fz - dz * fy)
    f = np.zeros(n_dofs(nel))
    f[3 * nodes + 1] = fy * moment / mom
    f[3 * nodes + 2] = fz * moment / mom
    return f


# --- named workloads --------------------------------------------------------

def column_2d_small(seed=1):
    """120x40 Q4 column, density 0.5 +- 0.1 smoothed (radius 2 el)."""
    nel = (120, 40)
    return dict(nel=nel, x=density_uniform_noise(nel, seed), fixed=clamp_mask(nel),
                F=axial_load(nel)[:, None])


def column_2d_large(seed=2):
    """960x320 Q4 column, smoothed random density with volume fraction 0.4."""
    nel = (960, 320)
    return dict(nel=nel, x=density_volume_fraction(nel, seed, 0.4, 8.0),
                fixed=clamp_mask(nel), F=axial_load(nel)[:, None])


def box_3d(nel=(192, 64, 64), seed=3, volfrac=0.3, sigma=4.0):
    """H8 box clamped at x = 0, axial pressure at x = nx, filtered density."""
    return dict(nel=tuple(nel), x=density_volume_fraction(tuple(nel), seed, volfrac, sigma),
                fixed=clamp_mask(tuple(nel)), F=axial_load(tuple(nel))[:, None])


def box_3d_four_cases(nel=(96, 48, 48), seed=4):
    """Four load cases: axial, shear y, shear z, torsion."""
    nel = tuple(nel)
    F = np.stack([axial_load(nel), shear_load(nel, 1), shear_load(nel, 2), torsion_load(nel)], axis=1)
    return dict(nel=nel, x=density_volume_fraction(nel, seed, 0.3, 4.0), fixed=clamp_mask(nel), F=F)


def small_instances_2d(count=32, seed=40):
    """Independent 2D Q4 instances of uneven sizes 64x32 ... 512x128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [(64, 32), (512, 128)]
    while len(sizes) < count:
        nx = int(rng.choice([64, 128, 256, 512]))
        ny = int(rng.choice([32, 64, 128]))
        if ny <= nx // 2:
            sizes.append((nx, ny))
    out = []
    for i, nel in enumerate(sizes):
        out.append(dict(nel=nel, x=density_volume_fraction(nel, 400 + i, 0.4, 8.0),
                        fixed=clamp_mask(nel), F=axial_load(nel)[:, None]))
    return out


def random_small(dim, nel, seed, lo=0.05, hi=1.0):
    """i.i.d. uniform densities in [lo, hi] (for property and parity tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=n_elems(nel))


def random_vectors(n, ncols, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=(n, ncols))
