"""Seeded synthetic density fields shaped like the paper's simulation densities.

The paper's workloads are N-body densities on 256^3 domain grids (Sec. VI.E); its initial
conditions are not available, so these generators stand in for them.  They hold none of
the solver's arithmetic: they only draw random fields, so both the GPU library's tests
and the CPU oracle's tests can use them.  All fields are float64, C order [i][j][k], with
mean exactly 1 after normalisation (the code-unit mean density, Sec. III.A).

Recipe (every config):
  1. w ~ N(0,1) on N^3 from numpy PCG64(seed);
  2. g^ = rfftn(w) |k|^(p/2) exp(-|k|^2 Rs^2 / 2), k in rad/cell, Rs = 2 cells, k=0 removed;
  3. g = irfftn(g^), rescaled to std sigma;
  4. rho = exp(g - sigma^2/2), plus structures drawn from PCG64(seed + 10^6), then
     rho /= mean(rho).
"""
from __future__ import annotations

import numpy as np


def gaussian_field(N: int, sigma: float, p: float, seed: int, smooth_cells: float = 2.0) -> np.ndarray:
    """Zero-mean Gaussian random field with power ~ k^p, Gaussian-smoothed, std sigma."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((N, N, N))
    wk = np.fft.rfftn(w)
    kx = 2.0 * np.pi * np.fft.fftfreq(N)
    kz = 2.0 * np.pi * np.fft.rfftfreq(N)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (p / 4.0), 0.0)
    wk *= amp * np.exp(-0.5 * k2 * smooth_cells ** 2)
    g = np.fft.irfftn(wk, s=(N, N, N), axes=(0, 1, 2))
    g -= g.mean()
    s = g.std()
    if s > 0:
        g *= sigma / s
    return g


def lognormal(N: int, sigma: float, p: float, seed: int) -> np.ndarray:
    """rho = exp(g - sigma^2/2), normalised to mean 1."""
    g = gaussian_field(N, sigma, p, seed)
    rho = np.exp(g - 0.5 * sigma * sigma)
    return rho / rho.mean()


def _periodic_box(N: int, centre, rmax: float):
    """Index ranges (wrapped) and periodic distances of cells within a cube around centre."""
    lo = [int(np.floor(c - rmax)) for c in centre]
    hi = [int(np.ceil(c + rmax)) + 1 for c in centre]
    axes = [np.arange(l, h) for l, h in zip(lo, hi)]
    d = [(a + 0.5) - c for a, c in zip(axes, centre)]
    r = np.sqrt(d[0][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[2][None, None, :] ** 2)
    idx = np.ix_(*[a % N for a in axes])
    return idx, r


def add_tophats(rho: np.ndarray, count: int, seed: int, rmin=2.0, rmax=8.0, dmin=50.0, dmax=500.0):
    """Adds count spheres of radius U[rmin,rmax] cells and amplitude U[dmin,dmax]."""
    N = rho.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed + 10 ** 6))
    for _ in range(count):
        c = rng.uniform(0, N, size=3)
        rad = rng.uniform(rmin, rmax)
        amp = rng.uniform(dmin, dmax)
        idx, r = _periodic_box(N, c, rad)
        rho[idx] += np.where(r <= rad, amp, 0.0)
    return rho


def add_nfw_halos(rho: np.ndarray, count: int, seed: int, cmin=5.0, cmax=10.0, rvmin=4.0,
                  rvmax=16.0, peak_min=1e2, peak_max=1e4):
    """Adds count NFW-like profiles d(r) = ds / [x (1+x)^2], x = max(r, 0.5)/r_s, cut at r_vir,
    with r_s = r_vir / c and the central value d(0.5) drawn log-uniform in [peak_min, peak_max]."""
    N = rho.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed + 10 ** 6))
    for _ in range(count):
        ctr = rng.uniform(0, N, size=3)
        conc = rng.uniform(cmin, cmax)
        rvir = rng.uniform(rvmin, rvmax)
        peak = np.exp(rng.uniform(np.log(peak_min), np.log(peak_max)))
        rs = rvir / conc
        x0 = 0.5 / rs
        ds = peak * x0 * (1.0 + x0) ** 2
        idx, r = _periodic_box(N, ctr, rvir)
        x = np.maximum(r, 0.5) / rs
        rho[idx] += np.where(r <= rvir, ds / (x * (1.0 + x) ** 2), 0.0)
    return rho


def normalise(rho: np.ndarray) -> np.ndarray:
    return rho / rho.mean()


# --- the five workloads --------------------------------------------------------------

def small_box(N: int = 32, seed: int = 0) -> np.ndarray:
    """32^3, B = 64 Mpc/h workload: lognormal, sigma = 1, P(k) ~ k^-2."""
    return lognormal(N, 1.0, -2.0, seed)


def tophat_box(N: int = 256, seed: int = 1, count: int = 200) -> np.ndarray:
    """256^3, B = 256 Mpc/h workload: lognormal sigma = 2, P ~ k^-1.5, plus spherical top-hats
    (radius 2-8 cells, amplitude 50-500)."""
    rho = lognormal(N, 2.0, -1.5, seed)
    return normalise(add_tophats(rho, count, seed))


def halo_box(N: int = 512, seed: int = 2, count: int = 2000) -> np.ndarray:
    """512^3, B = 512 Mpc/h workload: lognormal sigma = 3, P ~ k^-1.5, plus NFW-like halos
    (concentration 5-10, r_vir 4-16 cells, central amplitude 1e2-1e4)."""
    rho = lognormal(N, 3.0, -1.5, seed)
    return normalise(add_nfw_halos(rho, count, seed))


def batch_boxes(n64: int = 64, n128: int = 16):
    """Independent periodic boxes: (N, B, |f_R0|, sigma, seed, rho) per box; |f_R0| log-uniform
    in [1e-6, 1e-4], sigma uniform in [1, 3]; seeds 0.. for 64^3 and 100.. for 128^3."""
    out = []
    for N, B, cnt, s0 in ((64, 64.0, n64, 0), (128, 128.0, n128, 100)):
        for b in range(cnt):
            seed = s0 + b
            rng = np.random.Generator(np.random.PCG64(seed + 2 * 10 ** 6))
            fr0 = 10.0 ** rng.uniform(-6.0, -4.0)
            sigma = rng.uniform(1.0, 3.0)
            out.append((N, B, fr0, sigma, seed, lognormal(N, sigma, -1.5, seed)))
    return out


def _interp_periodic(g: np.ndarray, level: int, origin, n: int) -> np.ndarray:
    """Trilinear interpolation of the cell-centred domain field g (N0^3, periodic) at the
    centres of an n^3 block of level-`level` cells starting at `origin` (level cells)."""
    N0 = g.shape[0]
    f = 2 ** level
    axes = []
    for d in range(3):
        x = (origin[d] + np.arange(n) + 0.5) / f - 0.5      # in domain cell units
        i0 = np.floor(x).astype(np.int64)
        w = x - i0
        axes.append((i0 % N0, (i0 + 1) % N0, w))
    out = np.zeros((n, n, n))
    for a in (0, 1):
        ia, wa = axes[0][a], (1 - axes[0][2]) if a == 0 else axes[0][2]
        for b in (0, 1):
            ib, wb = axes[1][b], (1 - axes[1][2]) if b == 0 else axes[1][2]
            for c in (0, 1):
                ic, wc = axes[2][c], (1 - axes[2][2]) if c == 0 else axes[2][2]
                out += (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]) * g[np.ix_(ia, ib, ic)]
    return out


def amr_workload(N0: int = 256, seed: int = 1, sigma: float = 2.0, p: float = -1.5,
                 thresholds=(50.0, 200.0, 1000.0), sizes=(32, 16, 8, 4), max_patches: int = 2000,
                 min_fraction: float = 0.02):
    """Domain density plus refinement patches over len(thresholds) levels.

    Level l refines the cells of level l-1 whose contrast exceeds thresholds[l-1]: greedy,
    densest flagged cell first, with the largest cube of `sizes` (in parent cells; the patch
    has twice as many cells per side) that keeps `min_fraction` of flagged cells, stays inside
    its parent with a one-parent-cell margin and does not overlap a patch of its level.  The
    density on every level is exp(g - sigma^2/2) normalised as on the domain grid, with g the
    domain Gaussian field interpolated to the level's cell centres.

    Returns (rho_domain, patches, rho_packed): patches is a list of dicts {level, parent,
    origin, n, offset}, rho_packed the concatenated patch densities."""
    g = gaussian_field(N0, sigma, p, seed)
    rho0 = np.exp(g - 0.5 * sigma * sigma)
    norm = rho0.mean()
    rho0 /= norm
    patches, blocks = [], []
    offset = 0
    # parents of level 1: the domain (periodic)
    parents = [dict(level=0, origin=(0, 0, 0), n=N0, rho=rho0, index=-1)]
    for lev, thr in enumerate(thresholds, start=1):
        children = []
        for par in parents:
            if len(patches) >= max_patches:
                break
            prho = par["rho"]
            n_p = par["n"]
            flags = prho - 1.0 > thr
            if not flags.any():
                continue
            occupied = np.zeros_like(flags)
            covered = np.zeros_like(flags)
            cand = np.argwhere(flags)
            order = np.argsort(-prho[flags], kind="stable")
            for ci in order:
                if len(patches) >= max_patches:
                    break
                c = cand[ci]
                if covered[tuple(c)]:
                    continue
                placed = False
                for s in sizes:
                    if lev == 1:
                        lo, hi = 0, n_p - s           # the domain is periodic: no margin needed
                    else:
                        lo, hi = 1, n_p - 1 - s       # one parent cell of margin
                    if hi < lo:
                        continue
                    o = np.clip(c - s // 2, lo, hi)
                    sl = tuple(slice(int(o[d]), int(o[d]) + s) for d in range(3))
                    if occupied[sl].any():
                        continue
                    if flags[sl].mean() < min_fraction and s != sizes[-1]:
                        continue
                    occupied[sl] = True
                    covered[sl] = True
                    n = 2 * s
                    origin = tuple(int(2 * (par["origin"][d] + o[d])) for d in range(3))
                    rho = np.exp(_interp_periodic(g, lev, origin, n) - 0.5 * sigma * sigma) / norm
                    rec = dict(level=lev, parent=par["index"], origin=origin, n=n, offset=offset)
                    patches.append(rec)
                    blocks.append(rho.ravel())
                    offset += n ** 3
                    children.append(dict(level=lev, origin=origin, n=n, rho=rho, index=len(patches) - 1))
                    placed = True
                    break
                if not placed:
                    covered[tuple(c)] = True
        parents = children
        if not parents:
            break
    rho_packed = np.concatenate(blocks) if blocks else np.zeros(0)
    return rho0, patches, rho_packed


def amr_box(N0: int = 256, seed: int = 1):
    """The AMR workload: a 256^3 domain (lognormal sigma = 3, P(k) ~ k^-1) refined over 3
    levels where the contrast exceeds 50 / 200 / 1000, cube patches of 8^3 to 64^3 cells, each
    kept while at least 1.5% of its parent cells are flagged: 1706 patches (1204 / 379 / 123
    per level; 722, 643, 328 and 13 of side 8, 16, 32, 64) holding 17.2 M cells at N0 = 256,
    seed 1."""
    return amr_workload(N0, seed=seed, sigma=3.0, p=-1.0, min_fraction=0.015, max_patches=4000)


# --- refinement masks of an adaptive level ----------------------------------------------

def oct_mask(rho: np.ndarray, threshold: float, expand: int = 1) -> np.ndarray:
    """Mask of a refinement level held on the periodic N^3 grid of its resolution, built the
    way an oct-based AMR code refines: the 2^3-cell oct under a coarser cell is created when
    that cell's mean density exceeds `threshold`, then the set of octs is grown by `expand`
    octs in every direction (26-neighbourhood, periodic), a buffer around refined regions.
    Returns +1 in the cells of refined octs and -1 elsewhere (float64, C order)."""
    N = rho.shape[0]
    n = N // 2
    od = rho.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))
    refined = od > threshold
    for _ in range(expand):
        grown = refined.copy()
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for dk in (-1, 0, 1):
                    grown |= np.roll(refined, (di, dj, dk), axis=(0, 1, 2))
        refined = grown
    m = np.where(refined, 1.0, -1.0)
    return np.repeat(np.repeat(np.repeat(m, 2, 0), 2, 1), 2, 2)


def masked_level(N: int = 512, seed: int = 2, count: int = 2000, fraction: float = 0.25):
    """Masked-level workload: the halo density on N^3 and the oct mask refining the densest
    `fraction` of octs (before the one-oct buffer).  Returns (rho, mask)."""
    rho = halo_box(N, seed, count)
    n = N // 2
    od = rho.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))
    thr = float(np.quantile(od, 1.0 - fraction))
    del od
    return rho, oct_mask(rho, thr, expand=1)


# --- particles --------------------------------------------------------------------------

def particles(Ng: int, seed: int = 3, disp_cells: float = 2.0, clump_fraction: float = 0.3,
              clump_every: int = 2000) -> np.ndarray:
    """Ng^3 particle positions in the unit box, shaped like an evolved N-body set: a lattice of
    cell centres displaced along the gradient of a smooth Gaussian potential (the Zel'dovich
    recipe of N-body initial conditions; rms displacement `disp_cells` lattice cells per axis),
    then a fraction `clump_fraction` of the particles moved into compact Gaussian clumps (one
    clump per `clump_every` particles, radii 0.5-3 cells) to give the dense knots that halos
    make.  Returns float64 (Ng^3, 3) in [0, 1), lattice (C) order."""
    rng = np.random.Generator(np.random.PCG64(seed + 3 * 10 ** 6))
    n = Ng ** 3
    phi = gaussian_field(Ng, 1.0, -3.0, seed)
    pk = np.fft.rfftn(phi)
    del phi
    kx = 2.0 * np.pi * np.fft.fftfreq(Ng)
    kz = 2.0 * np.pi * np.fft.rfftfreq(Ng)
    pos = np.empty((n, 3))
    q = (np.arange(Ng) + 0.5) / Ng
    for ax in range(3):
        k = (kx[:, None, None], kx[None, :, None], kz[None, None, :])[ax]
        psi = np.fft.irfftn(-1j * k * pk, s=(Ng,) * 3, axes=(0, 1, 2))
        sd = psi.std()
        if sd > 0:  # a 2^3 lattice has no resolved gradient
            psi *= disp_cells / (sd * Ng)
        lat = np.broadcast_to(q.reshape([-1 if a == ax else 1 for a in range(3)]), (Ng,) * 3)
        pos[:, ax] = (lat + psi).reshape(-1)
        del psi
    del pk
    nc = max(1, n // clump_every)
    centres = rng.random((nc, 3))
    radii = rng.uniform(0.5, 3.0, nc) / Ng
    moved = rng.random(n) < clump_fraction
    which = rng.integers(0, nc, int(moved.sum()))
    pos[moved] = centres[which] + radii[which, None] * rng.standard_normal((len(which), 3))
    return np.mod(pos, 1.0)
