"""Grid and particle operations of the PM step in float64 NumPy (oracle;
test infrastructure only).

Conventions: periodic box of unit side, ``ng`` cells per side, cell size
h = 1/ng, cell (i,j,k) centred at ((i+1/2)h, (j+1/2)h, (k+1/2)h), fields in
C order with k fastest, positions as a (3, np) array in [0, 1).
"""
from __future__ import annotations

import numpy as np


def _cic_corners(pos, ng):
    """Base cell index and fractional offset of each particle per axis.

    The particle at x lies between the centres of cells i0 and i0+1 with
    u = x ng - 1/2, i0 = floor(u), f = u - i0; the Cloud-in-Cell weights are
    (1 - f) on i0 and f on i0+1 (Sec. 3.6.2 uses CIC assignment).
    """
    u = np.asarray(pos, dtype=np.float64) * ng - 0.5
    i0 = np.floor(u)
    f = u - i0
    return i0.astype(np.int64), f


def cic_deposit(pos, ng):
    """rho_c = (ng^3/np) sum_p W(x_p - x_c): density in units of the mean."""
    pos = np.asarray(pos, dtype=np.float64)
    npart = pos.shape[1]
    i0, f = _cic_corners(pos, ng)
    rho = np.zeros(ng**3)
    for dx in (0, 1):
        wx = f[0] if dx else 1.0 - f[0]
        ix = (i0[0] + dx) % ng
        for dy in (0, 1):
            wy = f[1] if dy else 1.0 - f[1]
            iy = (i0[1] + dy) % ng
            for dz in (0, 1):
                wz = f[2] if dz else 1.0 - f[2]
                iz = (i0[2] + dz) % ng
                idx = (ix * ng + iy) * ng + iz
                rho += np.bincount(idx, weights=wx * wy * wz, minlength=ng**3)
    return (rho * (ng**3 / npart)).reshape(ng, ng, ng)


def density_contrast(rho):
    """delta = rho - 1 - <rho - 1> (the source (rho - 1) of eq. phipsi_mod, made
    exactly mean-free)."""
    d = np.asarray(rho, dtype=np.float64) - 1.0
    return d - d.mean()


def laplacian7(u, h):
    """7-point discrete Laplacian on the periodic grid (Sec. 3.2.1)."""
    s = sum(np.roll(u, sh, axis=ax) for ax in range(3) for sh in (1, -1))
    return (s - 6.0 * u) / (h * h)


def laplacian7_eigenvalues(ng, h):
    """Eigenvalues -(4/h^2) sum_d sin^2(pi m_d/ng) of the periodic 7-point
    Laplacian on the rfftn grid."""
    m = np.fft.fftfreq(ng, d=1.0 / ng)
    mr = np.fft.rfftfreq(ng, d=1.0 / ng)
    sx = np.sin(np.pi * m / ng) ** 2
    sz = np.sin(np.pi * mr / ng) ** 2
    return -(4.0 / h**2) * (sx[:, None, None] + sx[None, :, None] + sz[None, None, :])


def poisson_fft(src, h):
    """Exact solution of lap_7 u = src - <src> on the periodic grid, <u> = 0."""
    ng = src.shape[0]
    lam = laplacian7_eigenvalues(ng, h)
    sh = np.fft.rfftn(src)
    lam[0, 0, 0] = 1.0
    uh = sh / lam
    uh[0, 0, 0] = 0.0
    return np.fft.irfftn(uh, s=src.shape, axes=(0, 1, 2))


def gradient5(u, h):
    """-grad u with the 5-point 4th-order stencil per axis (Sec. 3.5.2):
    D f_i = (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 h).
    Returns the acceleration field g = -D u as a (3, ng, ng, ng) array."""
    out = []
    for ax in range(3):
        fm2 = np.roll(u, 2, axis=ax)
        fm1 = np.roll(u, 1, axis=ax)
        fp1 = np.roll(u, -1, axis=ax)
        fp2 = np.roll(u, -2, axis=ax)
        out.append(-(fm2 - 8.0 * fm1 + 8.0 * fp1 - fp2) / (12.0 * h))
    return np.stack(out)


def cic_interpolate(field3, pos):
    """g_p = sum_c W(x_p - x_c) g_c with the same CIC kernel as the deposit."""
    ng = field3.shape[1]
    i0, f = _cic_corners(pos, ng)
    flat = field3.reshape(3, -1)
    out = np.zeros((3, np.asarray(pos).shape[1]))
    for dx in (0, 1):
        wx = f[0] if dx else 1.0 - f[0]
        ix = (i0[0] + dx) % ng
        for dy in (0, 1):
            wy = f[1] if dy else 1.0 - f[1]
            iy = (i0[1] + dy) % ng
            for dz in (0, 1):
                wz = f[2] if dz else 1.0 - f[2]
                iz = (i0[2] + dz) % ng
                idx = (ix * ng + iy) * ng + iz
                out += (wx * wy * wz) * flat[:, idx]
    return out


def power_spectrum(field, box, nbins=None):
    """Spherically averaged P(k) of a real periodic field (no window
    deconvolution): returns (k_centres, P, counts) with P = V <|delta_k|^2>."""
    ng = field.shape[0]
    fh = np.fft.rfftn(field) / ng**3
    kf = 2.0 * np.pi / box
    m = np.fft.fftfreq(ng, d=1.0 / ng)
    mr = np.fft.rfftfreq(ng, d=1.0 / ng)
    kk = kf * np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + mr[None, None, :] ** 2)
    wgt = np.full(fh.shape, 2.0)
    wgt[..., 0] = 1.0
    if ng % 2 == 0:
        wgt[..., -1] = 1.0
    nb = ng // 2 if nbins is None else nbins
    edges = kf * (np.arange(nb + 1) + 0.5)
    which = np.digitize(kk.ravel(), edges) - 1
    ok = (which >= 0) & (which < nb)
    p = (np.abs(fh) ** 2).ravel() * box**3
    cnt = np.bincount(which[ok], weights=wgt.ravel()[ok], minlength=nb)
    psum = np.bincount(which[ok], weights=(wgt.ravel() * p)[ok], minlength=nb)
    ksum = np.bincount(which[ok], weights=(wgt.ravel() * kk.ravel())[ok], minlength=nb)
    good = cnt > 0
    return ksum[good] / cnt[good], psum[good] / cnt[good], cnt[good]


def smoothed_ratio(k, p_num, p_den, sigma_k):
    """Boost R = p_num / p_den smoothed over the bins with a one-dimensional
    Gaussian filter of width sigma_k in k (normalised weights); sigma_k = 0
    returns R itself."""
    k = np.asarray(k, dtype=np.float64)
    r = np.asarray(p_num, dtype=np.float64) / np.asarray(p_den, dtype=np.float64)
    if sigma_k == 0.0:
        return r
    w = np.exp(-0.5 * ((k[None, :] - k[:, None]) / sigma_k) ** 2)
    return (w @ r) / w.sum(axis=1)
