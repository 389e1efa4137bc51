"""Seeded synthetic inputs: grids, transpose-buffer chunk geometry and fields.

This module holds the *inputs* only: it contains none of the codec's
arithmetic, imports nothing else from this package, and serves both the
HIP path and the CPU oracle in the tests.

Stand-in for the paper's data.  The paper compresses DYAMOND fields (Section
IV-A: temperature and ozone on a 2560 x 1281 grid, float32) which are not
available here.  Instead every field is a random spherical-harmonic series
truncated at total wavenumber L (T42 by default) with coefficient variance
proportional to (l+1)^-3, correlated 0.9 from one vertical level to the next,
sampled on Gauss-Legendre latitudes (the quadrature the paper's spectral
transform uses, Section II-A) and equally spaced longitudes, then
standardised over the whole 3-D field z and mapped to a physical-looking
variable: T = 280 + 15 z, u = v = 10 z, q = exp(z).

Grids.  Regular Gaussian grids (nlat x nlon) and reduced "octahedral" grids
in which latitude row j of each hemisphere (counted from the pole) has
20 + 4 j points, mirrored about the equator.

Buffers (the pencil-transposition send buffers of one GPU):
  * small    : one T field, 8 levels x 64 Gaussian latitudes x 128 longitudes.
  * z->lambda: one GPU's share of a 64-rank transposition at O1280-like
               resolution, 4 fields (u, v, T, q) x 137 levels x 64 rows x
               1612 points, cut into 64 equal per-destination chunks
               (destination d = field d // 16, row group d % 16).
  * lambda->theta: T on the O1280 reduced grid (2560 rows, 6,599,680 points
               per level) x 137 levels, cut by latitude into 256 destination
               chunks of whole 4-row groups (8 or 12 rows each).
  * large    : T on the O2560 reduced grid (5120 rows, 26,306,560 points per
               level) x 90 levels as one buffer.
  * serving  : requests of n values shaped (8, 64, n / 512), n log-uniform
               between 16,384 and 16,777,216 (64 KB to 64 MB of float32).
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

SEED_BASE = 260924294

FIELD_IDS = {"u": 0, "v": 1, "T": 2, "q": 3}


def seed_for(config: int, field: int) -> int:
    return SEED_BASE + 100 * config + field


# ---------------------------------------------------------------------------
# Chunk geometry (CSR form, the layout the library's plan call takes)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class ChunkSet:
    """Per-destination chunks of a float32 buffer.

    Chunk c: levels z = 0..levels[c]-1 at element offset
    chunk_base[c] + z * level_stride[c]; rows r = row_start[c]..row_start[c+1]-1
    at further element offset row_offset[r], each row_len[r] contiguous points.
    """
    chunk_base: np.ndarray    # int64 [nchunks]
    level_stride: np.ndarray  # int64 [nchunks]
    levels: np.ndarray        # int32 [nchunks]
    row_start: np.ndarray     # int32 [nchunks + 1]
    row_offset: np.ndarray    # int64 [nrows_total]
    row_len: np.ndarray       # int32 [nrows_total]
    buffer_elems: int         # size of the buffer the chunks index into

    def __post_init__(self):
        self.chunk_base = np.ascontiguousarray(self.chunk_base, np.int64)
        self.level_stride = np.ascontiguousarray(self.level_stride, np.int64)
        self.levels = np.ascontiguousarray(self.levels, np.int32)
        self.row_start = np.ascontiguousarray(self.row_start, np.int32)
        self.row_offset = np.ascontiguousarray(self.row_offset, np.int64)
        self.row_len = np.ascontiguousarray(self.row_len, np.int32)

    @property
    def nchunks(self) -> int:
        return int(self.chunk_base.size)

    def values(self) -> int:
        """Number of real (unpadded) values covered by all chunks."""
        tot = 0
        for c in range(self.nchunks):
            r0, r1 = self.row_start[c], self.row_start[c + 1]
            tot += int(self.levels[c]) * int(self.row_len[r0:r1].sum())
        return tot

    def subset(self, chunks) -> "ChunkSet":
        """A ChunkSet made of the listed chunks (same underlying buffer)."""
        chunks = list(chunks)
        rs = [0]
        offs, lens = [], []
        for c in chunks:
            r0, r1 = self.row_start[c], self.row_start[c + 1]
            offs.append(self.row_offset[r0:r1])
            lens.append(self.row_len[r0:r1])
            rs.append(rs[-1] + int(r1 - r0))
        return ChunkSet(self.chunk_base[chunks], self.level_stride[chunks], self.levels[chunks],
                        np.array(rs), np.concatenate(offs) if offs else np.zeros(0, np.int64),
                        np.concatenate(lens) if lens else np.zeros(0, np.int32),
                        self.buffer_elems)


def regular_chunkset(nz: int, ny: int, nx: int) -> ChunkSet:
    """A C-contiguous (nz, ny, nx) array as a single chunk."""
    return ChunkSet(np.array([0]), np.array([ny * nx]), np.array([nz]), np.array([0, ny]),
                    np.arange(ny, dtype=np.int64) * nx, np.full(ny, nx), nz * ny * nx)


def octahedral_row_lengths(n_half: int) -> np.ndarray:
    """Row lengths of a reduced octahedral grid with n_half rows per hemisphere."""
    north = 20 + 4 * np.arange(n_half, dtype=np.int64)
    return np.concatenate([north, north[::-1]])


def octahedral_row_offsets(lengths: np.ndarray) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)


def zlambda_chunkset(nfields=4, nlev=137, nrows=64, npts=1612, nchunks=64) -> ChunkSet:
    """One GPU's z->lambda send buffer f32[nfields][nlev][nrows][npts].

    Destination d gets field d // (nrows/4) and row group d % (nrows/4): all
    levels x 4 rows x npts points.
    """
    groups = nrows // 4
    assert nfields * groups == nchunks
    field_elems = nlev * nrows * npts
    base, rs, offs, lens = [], [0], [], []
    for d in range(nchunks):
        f, g = divmod(d, groups)
        base.append(f * field_elems + 4 * g * npts)
        offs.append(np.arange(4, dtype=np.int64) * npts)
        lens.append(np.full(4, npts))
        rs.append(rs[-1] + 4)
    return ChunkSet(np.array(base), np.full(nchunks, nrows * npts), np.full(nchunks, nlev),
                    np.array(rs), np.concatenate(offs), np.concatenate(lens),
                    nfields * field_elems)


def reduced_grid_chunkset(n_half: int, nlev: int, nchunks: int) -> ChunkSet:
    """A level-major f32[nlev][points] reduced-grid buffer cut by latitude.

    Rows are grouped in fours; chunk c takes row groups
    floor(G c / nchunks) .. floor(G (c+1) / nchunks) - 1 where G = 2 n_half / 4.
    """
    lengths = octahedral_row_lengths(n_half)
    offsets = octahedral_row_offsets(lengths)
    npoints = int(lengths.sum())
    G = lengths.size // 4
    assert lengths.size % 4 == 0 and nchunks <= G
    base, rs, offs, lens = [], [0], [], []
    for c in range(nchunks):
        g0, g1 = (G * c) // nchunks, (G * (c + 1)) // nchunks
        r0, r1 = 4 * g0, 4 * g1
        base.append(offsets[r0])
        offs.append(offsets[r0:r1] - offsets[r0])
        lens.append(lengths[r0:r1])
        rs.append(rs[-1] + (r1 - r0))
    return ChunkSet(np.array(base), np.full(nchunks, npoints), np.full(nchunks, nlev),
                    np.array(rs), np.concatenate(offs), np.concatenate(lens), nlev * npoints)


# Named buffers -------------------------------------------------------------

SMALL = dict(nlev=8, nlat=64, nlon=128)
ZLAMBDA = dict(nfields=4, nlev=137, nrows=64, npts=1612, nchunks=64, row0=1024, n_half=1280)
LTHETA = dict(n_half=1280, nlev=137, nchunks=256)
LARGE = dict(n_half=2560, nlev=90, nchunks=1)
# lambda->theta in Fourier space: rows 1024..1087 of O1280 (all hold 4116+ points,
# so every wavenumber up to the TCo1279 truncation), 137 levels, 16 destinations
FOURIER = dict(nlev=137, nrows=64, mmax=1279, ndest=16, row0=1024, n_half=1280)


def small_chunkset() -> ChunkSet:
    return regular_chunkset(SMALL["nlev"], SMALL["nlat"], SMALL["nlon"])


def ltheta_chunkset() -> ChunkSet:
    return reduced_grid_chunkset(LTHETA["n_half"], LTHETA["nlev"], LTHETA["nchunks"])


def fourier_buffer(L: int | None = None, nlev: int | None = None, nrows: int | None = None):
    """The Fourier-space lambda->theta share: (f32 planes [2][nlev][nrows][L+1],
    float64 planes) from T-field coefficients at Gauss latitudes row0.. of
    O1280 (seed of config 6)."""
    c = FOURIER
    L = c["mmax"] if L is None else L
    nlev = c["nlev"] if nlev is None else nlev
    nrows = c["nrows"] if nrows is None else nrows
    mu = gaussian_mu(2 * c["n_half"])[c["row0"]:c["row0"] + nrows]
    F = fourier_share(L, mu, nlev, seed_for(6, FIELD_IDS["T"]))
    return fourier_planes(F)


def large_chunkset() -> ChunkSet:
    return reduced_grid_chunkset(LARGE["n_half"], LARGE["nlev"], LARGE["nchunks"])


def pencil_message_dims(nodes: int, nlon=2560, nlat=1280, nlev=137):
    """Per-rank-pair sub-array of the paper's row transposition (Table 1 geometry):
    floor(n / sqrt(N)) along each axis of the nlon x nlat x nlev grid."""
    p = math.isqrt(nodes)
    assert p * p == nodes
    return nlon // p, nlat // p, nlev // p


# ---------------------------------------------------------------------------
# Random spherical-harmonic fields
# ---------------------------------------------------------------------------

def gaussian_mu(nlat: int) -> np.ndarray:
    """sin(latitude) of the Gauss-Legendre latitudes, north pole first."""
    x, _ = np.polynomial.legendre.leggauss(nlat)
    return x[::-1].copy()


def _legendre_m(L: int, m: int, mu: np.ndarray, pmm: np.ndarray) -> np.ndarray:
    """Orthonormal associated Legendre functions P_lm(mu), l = m..L, given P_mm."""
    out = np.zeros((mu.size, L - m + 1))
    out[:, 0] = pmm
    if L > m:
        out[:, 1] = math.sqrt(2 * m + 3) * mu * pmm
    for l in range(m + 2, L + 1):
        a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
        out[:, l - m] = a * (mu * out[:, l - m - 1] - b * out[:, l - m - 2])
    return out


def fourier_coefficients(L: int, mu: np.ndarray, nlev: int, seed: int, rho: float = 0.9,
                         zero_mean: bool = False) -> np.ndarray:
    """F[m, row, level] = sum_l a_lm(level) P_lm(mu_row), complex128.

    a_lm are complex Gaussian with E|a_lm|^2 = (l+1)^-3 (real for m = 0), and
    evolve from level to level as a <- rho a + sqrt(1 - rho^2) xi.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ls = np.arange(L + 1)
    sd = (ls + 1.0) ** -1.5
    F = np.zeros((L + 1, mu.size, nlev), np.complex128)
    # coefficients for all (l, m) and levels: A[m][l - m, level]
    A = []
    for m in range(L + 1):
        nl = L - m + 1
        A.append(np.zeros((nl, nlev), np.complex128))
    innov = math.sqrt(1.0 - rho * rho)
    for k in range(nlev):
        for m in range(L + 1):
            nl = L - m + 1
            s = sd[m:]
            if m == 0:
                xi = rng.standard_normal(nl) * s
            else:
                xi = (rng.standard_normal(nl) + 1j * rng.standard_normal(nl)) * s / math.sqrt(2)
            if zero_mean and m == 0:
                xi[0] = 0.0
            A[m][:, k] = xi if k == 0 else rho * A[m][:, k - 1] + innov * xi
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    pmm = np.full(mu.size, 1.0 / math.sqrt(4.0 * math.pi))
    for m in range(L + 1):
        if m > 0:
            pmm = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sin_t * pmm
        P = _legendre_m(L, m, mu, pmm)
        F[m] = P @ A[m]
    return F


def _ar1(x: np.ndarray, rho: float, gain: float) -> np.ndarray:
    """y[k] = rho y[k-1] + gain x[k] along axis 0, y[-1] = 0."""
    try:
        from scipy.signal import lfilter
        return lfilter([gain], [1.0, -rho], x, axis=0)
    except ImportError:  # pragma: no cover
        y = np.empty_like(x)
        y[0] = gain * x[0]
        for k in range(1, x.shape[0]):
            y[k] = rho * y[k - 1] + gain * x[k]
        return y


def fourier_share(L: int, mu: np.ndarray, nlev: int, seed: int, rho: float = 0.9) -> np.ndarray:
    """Fourier coefficients F[level, row, m] (m = 0..L, complex128) of a random
    spherical-harmonic field on the given latitude rows: what a row FFT of the
    grid field yields before the Legendre transform.

    a_lm are complex Gaussian with E|a_lm|^2 = (l+1)^-3 (real for m = 0),
    AR(1) from level to level with coefficient rho; generated one wavenumber
    at a time (innovations (l, level) per m), so any truncation L fits in
    memory.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    F = np.zeros((nlev, mu.size, L + 1), np.complex128)
    innov = math.sqrt(1.0 - rho * rho)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    pmm = np.full(mu.size, 1.0 / math.sqrt(4.0 * math.pi))
    for m in range(L + 1):
        if m > 0:
            pmm = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sin_t * pmm
        nl = L - m + 1
        sd = (np.arange(m, L + 1) + 1.0) ** -1.5
        if m == 0:
            xi = rng.standard_normal((nlev, nl)) * sd
        else:
            xi = (rng.standard_normal((nlev, nl)) + 1j * rng.standard_normal((nlev, nl))) \
                * (sd / math.sqrt(2))
        xi[0] /= innov  # A[0] = xi[0], then A[k] = rho A[k-1] + innov xi[k]
        A = _ar1(xi, rho, innov)
        P = _legendre_m(L, m, mu, pmm)          # (rows, l)
        F[:, :, m] = A @ P.T                    # (levels, rows)
    return F


def fourier_chunkset(nlev: int, nrows: int, mmax: int, ndest: int) -> ChunkSet:
    """The lambda->theta send buffer in Fourier space: f32[2][nlev][nrows][mmax+1]
    (real plane, then imaginary plane; m fastest).  Destination d gets the
    wavenumbers m0..m1-1, m0 = floor((mmax+1) d / ndest), of every row and
    level: its message is two chunks, the real one then the imaginary one."""
    M = mmax + 1
    plane = nlev * nrows * M
    base, rs, offs, lens = [], [0], [], []
    for d in range(ndest):
        m0, m1 = (M * d) // ndest, (M * (d + 1)) // ndest
        for part in (0, 1):
            base.append(part * plane + m0)
            offs.append(np.arange(nrows, dtype=np.int64) * M)
            lens.append(np.full(nrows, m1 - m0))
            rs.append(rs[-1] + nrows)
    n = 2 * ndest
    return ChunkSet(np.array(base), np.full(n, nrows * M), np.full(n, nlev), np.array(rs),
                    np.concatenate(offs), np.concatenate(lens), 2 * plane)


def fourier_planes(F: np.ndarray) -> np.ndarray:
    """Real and imaginary planes f32[2][nlev][nrows][mmax+1], scaled so that the
    whole buffer has unit RMS (the float64 planes before rounding are
    returned too)."""
    planes = np.stack([F.real, F.imag])
    planes = planes / math.sqrt(float(np.mean(planes * planes)))
    return planes.astype(np.float32), planes


def _irfft(c: np.ndarray, n: int) -> np.ndarray:
    try:
        import scipy.fft as sfft
        return sfft.irfft(c, n=n, axis=-1, workers=-1)
    except ImportError:  # pragma: no cover
        return np.fft.irfft(c, n=n, axis=-1)


def _row_values(Fm_row: np.ndarray, n: int, count: int) -> np.ndarray:
    """Values at longitudes 2 pi i / n, i < count, for all levels: (nlev, count).

    Fm_row: (L+1, nlev) complex Fourier coefficients of one latitude row.
    """
    L = Fm_row.shape[0] - 1
    if n > 2 * L:
        c = np.zeros((Fm_row.shape[1], n // 2 + 1), np.complex128)
        c[:, : L + 1] = Fm_row.T
        c[:, 0] = c[:, 0].real
        vals = _irfft(c, n) * n
        return vals[:, :count]
    lam = 2.0 * np.pi * np.arange(count) / n
    w = np.where(np.arange(L + 1) == 0, 1.0, 2.0)
    E = np.exp(1j * np.outer(np.arange(L + 1), lam))  # (L+1, count)
    return np.real((Fm_row.T * w) @ E)


def _finish(z: np.ndarray, kind: str) -> np.ndarray:
    if kind == "T":
        return 280.0 + 15.0 * z
    if kind in ("u", "v"):
        return 10.0 * z
    if kind == "q":
        return np.exp(z)
    raise ValueError(kind)


def field_on_rows(kind: str, mu_rows, row_lengths, counts, nlev: int, seed: int, L: int = 42,
                  out: np.ndarray | None = None, want_f64: bool = True):
    """A standardised random field on the given latitude rows.

    Row i has row_lengths[i] equally spaced longitudes of which the first
    counts[i] are kept.  Returns (f32 array [nlev, sum(counts)], f64 copy or
    None).  `out`, if given, is a float32 [nlev, sum(counts)] view to fill.
    """
    mu_rows = np.asarray(mu_rows, np.float64)
    counts = np.asarray(counts, np.int64)
    total = int(counts.sum())
    F = fourier_coefficients(L, mu_rows, nlev, seed, zero_mean=kind in ("u", "v"))
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    if want_f64:
        z = np.empty((nlev, total), np.float64)
        for i in range(mu_rows.size):
            z[:, offs[i]: offs[i] + counts[i]] = _row_values(F[:, i, :], int(row_lengths[i]),
                                                             int(counts[i]))
        z -= z.mean()
        z /= z.std()
        x64 = _finish(z, kind)
        x32 = x64.astype(np.float32)
        if out is not None:
            out[...] = x32
            x32 = out
        return x32, x64
    # float32-only path for very large buffers: two passes, stats in float64
    if out is None:
        out = np.empty((nlev, total), np.float32)
    s1 = 0.0
    s2 = 0.0
    for i in range(mu_rows.size):
        vals = _row_values(F[:, i, :], int(row_lengths[i]), int(counts[i]))
        s1 += float(vals.sum())
        s2 += float((vals * vals).sum())
        out[:, offs[i]: offs[i] + counts[i]] = vals
    n = float(nlev) * total
    mean = s1 / n
    std = math.sqrt(max(s2 / n - mean * mean, 1e-300))
    step = max(1, (1 << 24) // max(1, total))
    for k0 in range(0, nlev, step):
        blk = out[k0: k0 + step].astype(np.float64)
        blk = _finish((blk - mean) / std, kind)
        out[k0: k0 + step] = blk.astype(np.float32)
    return out, None


# Named buffers' data --------------------------------------------------------

def small_field(seed_offset: int = 0, L: int = 42):
    """T on the small regular grid: (f32 [8, 64, 128], f64 copy)."""
    nlev, nlat, nlon = SMALL["nlev"], SMALL["nlat"], SMALL["nlon"]
    mu = gaussian_mu(nlat)
    x32, x64 = field_on_rows("T", mu, np.full(nlat, nlon), np.full(nlat, nlon), nlev,
                             seed_for(1, FIELD_IDS["T"]) + seed_offset, L)
    return x32.reshape(nlev, nlat, nlon), x64.reshape(nlev, nlat, nlon)


def zlambda_fields(L: int = 42, want_f64: bool = True):
    """The z->lambda share f32[4][137][64][1612] (fields u, v, T, q)."""
    p = ZLAMBDA
    mu_all = gaussian_mu(2 * p["n_half"])
    lengths = octahedral_row_lengths(p["n_half"])
    rows = np.arange(p["row0"], p["row0"] + p["nrows"])
    x32 = np.empty((p["nfields"], p["nlev"], p["nrows"], p["npts"]), np.float32)
    x64 = np.empty(x32.shape, np.float64) if want_f64 else None
    for f, kind in enumerate(("u", "v", "T", "q")):
        a32, a64 = field_on_rows(kind, mu_all[rows], lengths[rows], np.full(rows.size, p["npts"]),
                                 p["nlev"], seed_for(2, f), L, want_f64=True)
        x32[f] = a32.reshape(p["nlev"], p["nrows"], p["npts"])
        if want_f64:
            x64[f] = a64.reshape(p["nlev"], p["nrows"], p["npts"])
    return x32, x64


def reduced_grid_field(n_half: int, nlev: int, config: int, L: int = 42,
                       nlev_take: int | None = None):
    """T on a reduced octahedral grid, f32 [nlev, points] (float32 only)."""
    mu = gaussian_mu(2 * n_half)
    lengths = octahedral_row_lengths(n_half)
    x32, _ = field_on_rows("T", mu, lengths, lengths, nlev, seed_for(config, FIELD_IDS["T"]), L,
                           want_f64=False)
    return x32


def ltheta_field(L: int = 42):
    return reduced_grid_field(LTHETA["n_half"], LTHETA["nlev"], 3, L)


def large_field(L: int = 42):
    return reduced_grid_field(LARGE["n_half"], LARGE["nlev"], 4, L)


def large_field_levels(nmade: int = 8, L: int = 42):
    """The first `nmade` levels (a multiple of 4) of the O2560 x 90 field.

    Generating all 90 levels takes minutes on the host; the large buffer is
    built by repeating these levels in order (see large_field_repeated), and
    since a 4x4x4 block spans 4 levels starting at a multiple of 4, no block
    straddles a repeat: every block has the generator's level-to-level
    statistics.
    """
    assert nmade % 4 == 0
    return reduced_grid_field(LARGE["n_half"], nmade, 4, L)


def large_field_repeated(levels: np.ndarray, nlev: int = LARGE["nlev"]) -> np.ndarray:
    """[nlev, points] float32: level k is levels[k % len(levels)]."""
    reps = -(-nlev // levels.shape[0])
    return np.ascontiguousarray(np.tile(levels, (reps, 1))[:nlev])


# ---------------------------------------------------------------------------
# Serving request stream
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    t_arrive: float  # seconds from the start of the stream
    op: int          # 0 compress, 1 decompress
    rate: int
    nx: int          # request shape (8, 64, nx); n = 512 nx values


def request_stream(count: int, mean_gap_s: float, seed: int = SEED_BASE + 5,
                   nmin: int = 16384, nmax: int = 16777216):
    """Poisson arrivals of mixed compress/decompress requests.

    Sizes are log-uniform in [nmin, nmax] values rounded to a multiple of
    2048; the op is compress or decompress with equal odds and the rate is
    uniform over {8, 16, 32}.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(mean_gap_s, count)
    t = np.cumsum(gaps) - gaps[0]
    n = np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))
    n = np.maximum(2048, np.round(n / 2048).astype(np.int64) * 2048)
    ops = rng.integers(0, 2, count)
    rates = rng.choice(np.array([8, 16, 32]), count)
    return [Request(float(t[i]), int(ops[i]), int(rates[i]), int(n[i] // 512))
            for i in range(count)]


def serving_pool(nx_max: int = 32768, L: int = 42):
    """One T field f32[8][64][nx_max] from which requests take (8, 64, nx) views."""
    mu = gaussian_mu(64)
    x32, _ = field_on_rows("T", mu, np.full(64, nx_max), np.full(64, nx_max), 8,
                           seed_for(5, FIELD_IDS["T"]), L, want_f64=False)
    return x32.reshape(8, 64, nx_max)


def cpu_count() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
