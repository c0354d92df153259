"""Seeded synthetic inputs for projected Krylov verification problems.

This module only *builds inputs*: system matrices (CSR or a 7-point stencil
descriptor), forcing vectors, initial-set generators, output rows and unsafe
intervals.  It holds none of the verification method's arithmetic, so both the
CPU oracle (``oracle/``) and the GPU library's tests and benchmark can draw
their inputs from here without sharing any of the method.

Problem statement followed (paper, Section 2 "Affine Verification Review"):
dynamics x' = A x + b, an initial set, an unsafe set, a step dt and a number
of steps S.  Initial sets are boxes in an initial space x0 = E z (Section 3.2):
each generator is a sparse column of E (a set of index ranges with values)
with z_j in [zc_j - r_j, zc_j + r_j].  Outputs y = C x use sparse rows of C
(Section 3.1).  An optional dense ``center`` vector is a fixed (coefficient 1)
part of x0 that is not in the generators' span.

Grid ordering for 3D problems: index = (ix * ny + iy) * nz + iz (x slowest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Segments", "Generator", "Problem",
    "segments_from_ranges", "box_segments", "csr_stencil7",
    "harmonic_oscillator", "heat1d", "heat3d_csr", "heat3d_stencil", "heat3d_paper", "csr_heat_insulated",
    "heat3d_paper_stencil", "csr_stencil7_faces",
    "random_symmetric", "small_heat3d", "conv_diff3d", "heat3d_many_gens",
    "segments_of_dense", "heat3d_many_inputs",
]


@dataclass
class Segments:
    """A sparse vector given as disjoint, sorted half-open index ranges
    [lo[i], hi[i]) that each carry one value w[i]."""
    lo: np.ndarray
    hi: np.ndarray
    w: np.ndarray

    def __post_init__(self):
        self.lo = np.ascontiguousarray(self.lo, dtype=np.int64)
        self.hi = np.ascontiguousarray(self.hi, dtype=np.int64)
        self.w = np.ascontiguousarray(self.w, dtype=np.float64)
        if not (self.lo.shape == self.hi.shape == self.w.shape):
            raise ValueError("segment arrays differ in length")
        if np.any(self.hi <= self.lo):
            raise ValueError("empty or inverted segment")
        if self.lo.size > 1 and np.any(self.lo[1:] < self.hi[:-1]):
            raise ValueError("segments must be sorted and disjoint")

    @property
    def nseg(self) -> int:
        return int(self.lo.size)

    @property
    def count(self) -> int:
        return int((self.hi - self.lo).sum())

    def dense(self, n: int) -> np.ndarray:
        v = np.zeros(n)
        for a, b, w in zip(self.lo, self.hi, self.w):
            v[a:b] = w
        return v


@dataclass
class Generator:
    """One column of E as index ranges, with its box z in [zc-radius, zc+radius]."""
    seg: Segments
    zc: float
    radius: float


@dataclass
class Problem:
    name: str
    n: int
    kind: str                      # "csr" or "stencil7"
    symmetric: bool
    gens: List[Generator]
    C: List[Segments]              # o output rows
    unsafe: np.ndarray             # (o, 2): row r is unsafe when y_r in [lo, hi]
    k: int
    dt: float
    steps: int                     # S; time points s = 0..S
    b: Optional[np.ndarray] = None
    center: Optional[np.ndarray] = None
    # CSR
    rowptr: Optional[np.ndarray] = None
    colidx: Optional[np.ndarray] = None
    vals: Optional[np.ndarray] = None
    # 7-point stencil with zero (Dirichlet) values outside the grid
    grid: Optional[Tuple[int, int, int]] = None
    coef: Optional[Tuple[float, float, float, float]] = None   # (c0, cx, cy, cz)
    seed: int = 0
    note: str = ""
    meta: dict = field(default_factory=dict)
    b_seg: Optional[Segments] = None    # forcing as index ranges (instead of a dense b)
    # stencil face conditions: "dirichlet" (zero outside the grid) or "insulated"
    # (no flux: a missing neighbour's coefficient returns to the diagonal), and
    # a term added to the diagonal of the last x plane (exchange through x = 1)
    bc: str = "dirichlet"
    exchange: float = 0.0

    @property
    def has_forcing(self) -> bool:
        return self.b is not None or self.b_seg is not None

    def forcing(self) -> Optional[np.ndarray]:
        """Dense forcing vector b (None when there is none)."""
        if self.b is not None:
            return np.asarray(self.b, np.float64)
        if self.b_seg is not None:
            return self.b_seg.dense(self.n)
        return None

    @property
    def o(self) -> int:
        return len(self.C)

    @property
    def nnz(self) -> int:
        return 0 if self.colidx is None else int(self.colidx.size)

    def csr(self):
        """(rowptr, colidx, vals); a stencil problem is expanded to CSR."""
        if self.kind == "csr":
            return self.rowptr, self.colidx, self.vals
        nx, ny, nz = self.grid
        if self.bc == "dirichlet" and self.exchange == 0.0:
            return csr_stencil7(nx, ny, nz, *self.coef)
        return csr_stencil7_faces(nx, ny, nz, *self.coef, insulated=self.bc == "insulated", exchange=self.exchange)


def segments_from_ranges(ranges, values=1.0) -> Segments:
    ranges = sorted(ranges)
    vals = np.broadcast_to(np.asarray(values, dtype=np.float64), (len(ranges),))
    return Segments(np.array([r[0] for r in ranges]), np.array([r[1] for r in ranges]), np.array(vals))


def segments_of_dense(v) -> Segments:
    """The same vector as index ranges: each maximal run of equal nonzero
    consecutive entries becomes one range (a change of format only)."""
    v = np.asarray(v, np.float64)
    lo, hi, w = [], [], []
    i, n = 0, v.size
    while i < n:
        if v[i] == 0.0:
            i += 1
            continue
        j = i + 1
        while j < n and v[j] == v[i]:
            j += 1
        lo.append(i); hi.append(j); w.append(v[i])
        i = j
    return Segments(np.array(lo, np.int64), np.array(hi, np.int64), np.array(w))


def box_segments(grid, box, value=1.0) -> Segments:
    """Index ranges of the cells of a 3D box ((x0,x1),(y0,y1),(z0,z1)), half
    open, in a grid (nx, ny, nz) ordered x slowest.  Runs along z are merged
    when the box spans the whole z (and y) extent."""
    nx, ny, nz = grid
    (x0, x1), (y0, y1), (z0, z1) = box
    assert 0 <= x0 < x1 <= nx and 0 <= y0 < y1 <= ny and 0 <= z0 < z1 <= nz
    if z0 == 0 and z1 == nz and y0 == 0 and y1 == ny:
        lo = np.array([x0 * ny * nz]); hi = np.array([x1 * ny * nz])
    elif z0 == 0 and z1 == nz:
        xs = np.arange(x0, x1)
        lo = (xs * ny + y0) * nz
        hi = (xs * ny + y1) * nz
    else:
        xs, ys = np.meshgrid(np.arange(x0, x1), np.arange(y0, y1), indexing="ij")
        base = ((xs * ny + ys) * nz).ravel()
        lo = base + z0
        hi = base + z1
    return Segments(lo, hi, np.full(lo.size, float(value)))


def csr_stencil7(nx, ny, nz, c0, cx, cy, cz):
    """CSR (int64 rowptr, int32 colidx, float64 values) of the 7-point
    stencil with zero values outside the grid; columns ascending per row."""
    n = nx * ny * nz
    if n >= 2**31:
        raise ValueError("CSR expansion limited to n < 2^31 (int32 columns)")
    idx = np.arange(n, dtype=np.int64)
    iz = idx % nz
    iy = (idx // nz) % ny
    ix = idx // (ny * nz)
    offs = [(-ny * nz, ix > 0, cx), (-nz, iy > 0, cy), (-1, iz > 0, cz), (0, None, c0),
            (1, iz < nz - 1, cz), (nz, iy < ny - 1, cy), (ny * nz, ix < nx - 1, cx)]
    cols = np.empty((n, 7), dtype=np.int64)
    vals = np.empty((n, 7), dtype=np.float64)
    mask = np.empty((n, 7), dtype=bool)
    for j, (d, ok, c) in enumerate(offs):
        cols[:, j] = idx + d
        vals[:, j] = c
        mask[:, j] = True if ok is None else ok
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colidx = cols[mask].astype(np.int32)
    v = vals[mask]
    return rowptr, colidx, v


# ---------------------------------------------------------------------------
# The paper's worked example (Section 2.2 "Timed Harmonic Oscillator Example")
# ---------------------------------------------------------------------------

def harmonic_oscillator() -> Problem:
    """x' = y, y' = -x, t' = 1 (the t equation carries the affine term);
    x0 = -5, y0 in [0, 1], t0 = 0; unsafe when x = 4; step pi/4 up to pi."""
    rowptr = np.array([0, 1, 2, 2], dtype=np.int64)
    colidx = np.array([1, 0], dtype=np.int32)
    vals = np.array([1.0, -1.0])
    b = np.array([0.0, 0.0, 1.0])
    gen = Generator(segments_from_ranges([(1, 2)]), zc=0.5, radius=0.5)
    center = np.array([-5.0, 0.0, 0.0])
    C = [segments_from_ranges([(0, 1)])]
    unsafe = np.array([[4.0, 4.0]])
    return Problem("harmonic", 3, "csr", False, [gen], C, unsafe, k=3, dt=math.pi / 4, steps=4,
                   b=b, center=center, rowptr=rowptr, colidx=colidx, vals=vals,
                   note="paper Section 2.2 worked example")


# ---------------------------------------------------------------------------
# 1D heat equation, n = 200 (tridiagonal (1,-2,1)/h^2, Dirichlet ends)
# ---------------------------------------------------------------------------

def heat1d(n=200, k=30, dt=1e-4, steps=1000, seed=1) -> Problem:
    h = 1.0 / (n + 1)
    rowptr, colidx, vals = csr_stencil7(1, 1, n, -2.0 / h**2, 0.0, 0.0, 1.0 / h**2)
    rng = np.random.default_rng(seed)
    xc = rng.uniform(0.0, 1.0, size=10)
    gens = [Generator(segments_from_ranges([(j, j + 1)]), zc=float(xc[j]), radius=0.05)
            for j in range(10)]
    # output: mean of x_90..x_110 (1-based), i.e. indices 89..109
    C = [segments_from_ranges([(89, 110)], 1.0 / 21.0)]
    unsafe = np.array([[0.9, math.inf]])
    return Problem("heat1d", n, "csr", True, gens, C, unsafe, k=k, dt=dt, steps=steps,
                   rowptr=rowptr, colidx=colidx, vals=vals, seed=seed,
                   note="1D heat, box radius 0.05 on x_1..x_10, mean(x_90..x_110) >= 0.9 unsafe")


# ---------------------------------------------------------------------------
# 3D heat equation (Dirichlet faces), diffusivity D, h = 1/(m+1)
# ---------------------------------------------------------------------------

def _heat3d_parts(m, D, seed, forcing_cube=10, forcing=0.1):
    h = 1.0 / (m + 1)
    c = D / h**2
    coef = (-6.0 * c, c, c, c)
    forcing_cube = min(forcing_cube, m)
    rng = np.random.default_rng(seed)
    off = rng.integers(0, m - forcing_cube + 1, size=3)
    fbox = tuple((int(o), int(o) + forcing_cube) for o in off)
    b = box_segments((m, m, m), fbox, forcing).dense(m**3)
    return coef, b, fbox


def heat3d_csr(m=100, D=0.01, k=40, dt=0.02, steps=2000, seed=2, unsafe_scale=None) -> Problem:
    """3D heat on an m^3 grid stored as CSR, forcing b = 0.1 on a seeded
    10^3 sub-cube (state augmentation), one box generator over the [0,10)^3
    corner at 1.0 +- 0.1, outputs = means over the generator cube, the
    forcing cube and the central cube."""
    n = m**3
    coef, b, fbox = _heat3d_parts(m, D, seed)
    rowptr, colidx, vals = csr_stencil7(m, m, m, *coef)
    g = min(10, m)
    gbox = ((0, g), (0, g), (0, g))
    gens = [Generator(box_segments((m, m, m), gbox, 1.0), zc=1.0, radius=0.1)]
    cc = max(m // 2 - g // 2, 0)
    cbox = ((cc, cc + g), (cc, cc + g), (cc, cc + g))
    C = []
    for bx in (gbox, fbox, cbox):
        cells = int(np.prod([hi - lo for lo, hi in bx]))
        C.append(box_segments((m, m, m), bx, 1.0 / cells))
    # unsafe thresholds: region means reaching these values are unsafe.
    thr = np.array([1.2, 0.5, 0.5]) if unsafe_scale is None else np.asarray(unsafe_scale, float)
    unsafe = np.stack([thr, np.full(3, math.inf)], axis=1)
    return Problem("heat3d_csr", n, "csr", True, gens, C, unsafe, k=k, dt=dt, steps=steps,
                   b=b, rowptr=rowptr, colidx=colidx, vals=vals, seed=seed,
                   meta={"m": m, "forcing_box": fbox, "gen_box": gbox, "center_box": cbox, "coef": coef},
                   note="3D heat CSR with affine forcing")


def csr_stencil7_faces(nx, ny, nz, c0, cx, cy, cz, insulated=False, exchange=0.0):
    """CSR of the 7-point stencil with face conditions: with `insulated`, a
    row's diagonal is c0 plus the coefficient of each missing neighbour
    (added in the order x-, x+, y-, y+, z-, z+); `exchange` is then added on
    the last x plane."""
    rowptr, colidx, vals = csr_stencil7(nx, ny, nz, c0, cx, cy, cz)
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    iz = idx % nz
    iy = (idx // nz) % ny
    ix = idx // (ny * nz)
    d = np.full(n, float(c0))
    if insulated:
        for miss, c in ((ix == 0, cx), (ix == nx - 1, cx), (iy == 0, cy), (iy == ny - 1, cy),
                        (iz == 0, cz), (iz == nz - 1, cz)):
            d = np.where(miss, d + c, d)
    d = np.where(ix == nx - 1, d + exchange, d)
    rows = np.repeat(idx, np.diff(rowptr))
    on_diag = colidx.astype(np.int64) == rows
    vals = vals.copy()
    vals[on_diag] = d[rows[on_diag]]
    return rowptr, colidx, vals


def heat3d_paper_stencil(m=1000, D=0.01, exchange=0.5, k=5932, dt=0.02, steps=1000) -> Problem:
    """heat3d_paper as a matrix-free stencil (insulated faces, exchange on
    the x = 1 face), for grids too large to store; the same operator up to
    the rounding of the diagonal."""
    p = heat3d_paper(m=min(m, 2), D=D, exchange=exchange)        # shapes only
    n = m**3
    h = 1.0 / (m + 1)
    c = D / h**2
    gbox, cbox, cells = _paper_heat_regions(m)
    gens = [Generator(box_segments((m, m, m), gbox, 1.0), zc=1.0, radius=0.1)]
    C = [box_segments((m, m, m), cbox, 1.0 / cells)]
    return Problem("heat3d_paper_stencil", n, "stencil7", True, gens, C, p.unsafe, k=k, dt=dt, steps=steps,
                   grid=(m, m, m), coef=(-6.0 * c, c, c, c), bc="insulated", exchange=-c * h * exchange,
                   meta={"m": m, "gen_box": gbox, "center_box": cbox, "c": c, "h": h, "exchange": exchange},
                   note="3D heat as stated in the paper, matrix-free")


def _paper_heat_regions(m):
    """Index boxes of the heated region x in [0, 0.4], y in [0, 0.2],
    z in [0, 0.1] (the grid points (i + 1) h with h = 1 / (m + 1) inside it,
    at least one per axis) and of the points around the centre (0.5, 0.5,
    0.5): the centre point itself for odd m, the 8 around it for even m."""
    ext = [max(int(math.floor(f * (m + 1) + 1e-9)), 1) for f in (0.4, 0.2, 0.1)]
    gbox = ((0, ext[0]), (0, ext[1]), (0, ext[2]))
    mid = [m // 2 - 1, m // 2] if m % 2 == 0 else [m // 2]
    cbox = tuple((mid[0], mid[-1] + 1) for _ in range(3))
    return gbox, cbox, len(mid) ** 3


def csr_heat_insulated(m, c, exchange_diag):
    """CSR of the cell-centred 7-point heat operator on an m^3 grid with
    insulated faces (no flux: a face without a neighbour adds neither the
    neighbour nor its -c to the diagonal) plus `exchange_diag` added to the
    diagonal of the cells on the x = 1 face (ix = m - 1).  Symmetric."""
    n = m**3
    if n >= 2**31:
        raise ValueError("CSR expansion limited to n < 2^31 (int32 columns)")
    idx = np.arange(n, dtype=np.int64)
    iz = idx % m
    iy = (idx // m) % m
    ix = idx // (m * m)
    nbrs = [(-m * m, ix > 0), (-m, iy > 0), (-1, iz > 0), (1, iz < m - 1), (m, iy < m - 1), (m * m, ix < m - 1)]
    diag = -c * sum(ok.astype(np.float64) for _, ok in nbrs) + np.where(ix == m - 1, exchange_diag, 0.0)
    cols = np.empty((n, 7), dtype=np.int64)
    vals = np.empty((n, 7), dtype=np.float64)
    mask = np.empty((n, 7), dtype=bool)
    order = nbrs[:3] + [(0, None)] + nbrs[3:]
    for j, (d, ok) in enumerate(order):
        cols[:, j] = idx + d
        vals[:, j] = diag if ok is None else c
        mask[:, j] = True if ok is None else ok
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=rowptr[1:])
    return rowptr, cols[mask].astype(np.int32), vals[mask]


def heat3d_paper(m=100, D=0.01, exchange=0.5, k=1024, dt=0.02, steps=1000) -> Problem:
    """The 3D heat benchmark as the paper states it (Section 5.3): unit cube,
    all faces insulated except x = 1, which exchanges heat with a 0-degree
    ambient at constant 0.5; u_t = D (u_xx + u_yy + u_zz), D = 0.01;
    initially 0.9..1.1 on x in [0, 0.4], y in [0, 0.2], z in [0, 0.1] and 0
    elsewhere; output = the temperature at the centre point; T = 20 with
    dt = 0.02.  Semi-discretised on the m^3 grid points (i + 1) h,
    h = 1 / (m + 1), by second differences c (u_j - u_i), c = D / h^2, with
    no flux through insulated faces (a missing neighbour contributes nothing)
    and, on the x = 1 face, the exchange flux D * exchange * u through a face
    of area h^2 into a volume h^3, i.e. -c h exchange on those points'
    diagonal.  This spacing reproduces the paper's |A t| at t = 50 for m = 100
    (Section 4.2).  The centre point is the mean of the 8 points around it
    (m even) or the centre point (m odd).  k is the cap of an
    error-controlled Krylov dimension."""
    n = m**3
    h = 1.0 / (m + 1)
    c = D / h**2
    rowptr, colidx, vals = csr_heat_insulated(m, c, -c * h * exchange)
    gbox, cbox, cells = _paper_heat_regions(m)
    gens = [Generator(box_segments((m, m, m), gbox, 1.0), zc=1.0, radius=0.1)]
    C = [box_segments((m, m, m), cbox, 1.0 / cells)]
    unsafe = np.array([[1.0, math.inf]])
    return Problem("heat3d_paper", n, "csr", True, gens, C, unsafe, k=k, dt=dt, steps=steps,
                   rowptr=rowptr, colidx=colidx, vals=vals,
                   meta={"m": m, "gen_box": gbox, "center_box": cbox, "c": c, "h": h, "exchange": exchange},
                   note="3D heat as stated in the paper: insulated faces, exchange at x = 1, centre-point output")


def small_heat3d(m=12, D=0.01, k=20, dt=0.02, steps=200, seed=7) -> Problem:
    """A small version of heat3d_csr for fast parity runs."""
    p = heat3d_csr(m=m, D=D, k=k, dt=dt, steps=steps, seed=seed)
    p.name = "small_heat3d"
    return p


def heat3d_many_inputs(m=100, D=0.01, k=40, dt=0.02, steps=1000, seed=5, floor=0.01) -> Problem:
    """An initial space wider than the output space (i = 8 > o = 1), the case
    the transposed simulation of Section 4.1 is for: 3D heat on an m^3 grid
    (CSR, Dirichlet), forcing 0.1 on a seeded 10^3 sub-cube given as index
    ranges, six box generators over disjoint seeded 8^3 cubes (z = 1.0 +- 0.1
    each), a fixed initial part 0.5 on a seeded 12^3 warm cube (the center,
    also as index ranges), and one output: the mean over the warm cube,
    unsafe when it cools to `floor` or below."""
    n = m**3
    coef, _, fbox = _heat3d_parts(m, D, seed)
    bseg = box_segments((m, m, m), fbox, 0.1)
    rowptr, colidx, vals = csr_stencil7(m, m, m, *coef)
    rng = np.random.default_rng(seed + 1)
    g = min(8, m)
    cells = max(m // g, 1)
    picks = rng.choice(cells**3, size=min(6, cells**3), replace=False)
    gens = []
    for pk in sorted(int(x) for x in picks):
        cx, cy, cz = pk // (cells * cells), (pk // cells) % cells, pk % cells
        gb = ((cx * g, cx * g + g), (cy * g, cy * g + g), (cz * g, cz * g + g))
        gens.append(Generator(box_segments((m, m, m), gb, 1.0), zc=1.0, radius=0.1))
    wc = min(12, m)
    woff = int(rng.integers(0, m - wc + 1))
    wbox = ((woff, woff + wc),) * 3
    center_seg = box_segments((m, m, m), wbox, 0.5)
    C = [box_segments((m, m, m), wbox, 1.0 / wc**3)]
    unsafe = np.array([[-math.inf, float(floor)]])
    return Problem("heat3d_many_inputs", n, "csr", True, gens, C, unsafe, k=k, dt=dt, steps=steps,
                   b_seg=bseg, center=center_seg.dense(n), rowptr=rowptr, colidx=colidx, vals=vals, seed=seed,
                   meta={"m": m, "forcing_box": fbox, "warm_box": wbox},
                   note="3D heat, eight initial-space columns, one output")


def heat3d_many_gens(m=100, g=5, ngen=256, D=0.01, k=40, dt=0.02, steps=1000, seed=6, floor=0.01) -> Problem:
    """An initial space of hundreds of columns and one output (i >> o, the
    transposed route's case): the system, forcing and warm cube of
    heat3d_many_inputs, with `ngen` box generators on distinct seeded g^3
    cells of the grid (1.0 +- 0.1 each) instead of six."""
    base = heat3d_many_inputs(m=m, D=D, k=k, dt=dt, steps=steps, seed=seed, floor=floor)
    cells = m // g
    rng = np.random.default_rng(seed + 2)
    picks = rng.choice(cells**3, size=min(ngen, cells**3), replace=False)
    gens = []
    for pk in sorted(int(x) for x in picks):
        cx, cy, cz = pk // (cells * cells), (pk // cells) % cells, pk % cells
        gb = ((cx * g, cx * g + g), (cy * g, cy * g + g), (cz * g, cz * g + g))
        gens.append(Generator(box_segments((m, m, m), gb, 1.0), zc=1.0, radius=0.1))
    base.gens = gens
    base.name = "heat3d_many_gens"
    base.note = f"3D heat, {len(gens) + 2} initial-space columns, one output"
    return base


def heat3d_stencil(m=1000, D=0.01, k=20, dt=0.01, steps=500, seed=4) -> Problem:
    """Matrix-free 3D heat (7-point stencil descriptor), forcing 0.1 on a
    seeded 100^3 sub-cube, generator = heated region x in [0,0.4],
    y in [0,0.2], z in [0,0.1] (paper Section 5.3) at 1.0 +- 0.1, outputs =
    the grid center point and the mean over the heated region."""
    n = m**3
    h = 1.0 / (m + 1)
    c = D / h**2
    coef = (-6.0 * c, c, c, c)
    rng = np.random.default_rng(seed)
    fc = max(m // 10, 1)
    off = rng.integers(0, m - fc + 1, size=3)
    fbox = tuple((int(o), int(o) + fc) for o in off)
    bseg = box_segments((m, m, m), fbox, 0.1)
    gbox = ((0, max(int(round(0.4 * m)), 1)), (0, max(int(round(0.2 * m)), 1)),
            (0, max(int(round(0.1 * m)), 1)))
    gseg = box_segments((m, m, m), gbox, 1.0)
    gens = [Generator(gseg, zc=1.0, radius=0.1)]
    mid = m // 2
    cpt = ((mid * m + mid) * m + mid)
    C = [segments_from_ranges([(cpt, cpt + 1)]), box_segments((m, m, m), gbox, 1.0 / gseg.count)]
    unsafe = np.array([[0.5, math.inf], [1.2, math.inf]])
    return Problem("heat3d_stencil", n, "stencil7", True, gens, C, unsafe, k=k, dt=dt, steps=steps,
                   b_seg=bseg, grid=(m, m, m), coef=coef, seed=seed,
                   meta={"m": m, "forcing_box": fbox, "gen_box": gbox},
                   note="matrix-free 3D heat with affine forcing")


def _clip_box(box, lo, hi):
    return tuple((max(a, l), min(b, h)) for (a, b), l, h in zip(box, lo, hi))


def heat3d_stencil_subgrid(full: Problem, role: str, k: Optional[int] = None):
    """One run of a heat3d_stencil problem ("gen": the generator over the
    heated region; "affine": the forcing) restated on a small sub-grid with
    the same result.  After j Krylov steps from a start vector supported in
    a box, every basis vector is supported within grid distance j of that
    box (A is a 7-point stencil), so the run equals the same run on the
    sub-grid spanned by the box dilated by k + 1 cells (its own zero faces
    are never reached), with the outputs restricted to that sub-grid.
    Returns (sub_problem or None, rows): rows[q] is the sub-problem's output
    index of full output row q, or None when row q lies outside the sub-grid
    (its basis entries are exactly zero); sub_problem is None when no
    output row meets the sub-grid."""
    m = full.meta["m"]
    k = full.k if k is None else k
    start_box = full.meta["gen_box"] if role == "gen" else full.meta["forcing_box"]
    lo = [max(a - (k + 1), 0) for a, _ in start_box]
    hi = [min(b + (k + 1), m) for _, b in start_box]
    grid = tuple(h - l for l, h in zip(lo, hi))

    def shift(box):
        return tuple((a - l, b - l) for (a, b), l in zip(box, lo))

    mid = m // 2
    gcount = int(np.prod([b - a for a, b in full.meta["gen_box"]]))
    C, rows = [], []
    for q, box in enumerate([((mid, mid + 1),) * 3, full.meta["gen_box"]]):
        cb = _clip_box(box, lo, hi)
        if all(b > a for a, b in cb):
            rows.append(len(C))
            C.append(box_segments(grid, shift(cb), 1.0 if q == 0 else 1.0 / gcount))
        else:
            rows.append(None)
    if not C:
        return None, rows
    sb = shift(start_box)
    gens, bseg = [], None
    if role == "gen":
        g = full.gens[0]
        gens = [Generator(box_segments(grid, sb, 1.0), zc=g.zc, radius=g.radius)]
    else:
        bseg = box_segments(grid, sb, 0.1)
    sub = Problem("heat3d_stencil_subgrid", int(np.prod(grid)), "stencil7", True, gens, C,
                  np.array([[math.inf, math.inf]] * len(C)), k=k, dt=full.dt, steps=full.steps,
                  b_seg=bseg, grid=grid, coef=full.coef, meta={"offset": tuple(lo), "role": role})
    return sub, rows


# ---------------------------------------------------------------------------
# Small random problems for parity edge cases
# ---------------------------------------------------------------------------

def random_symmetric(n=300, nnz_per_row=5, k=12, steps=50, dt=0.05, ngen=3, o=2, seed=11,
                     affine=True, center=False) -> Problem:
    """A random sparse symmetric negative-definite-ish matrix (symmetrised
    random pattern minus a diagonal shift), random index-range generators
    and output rows."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), nnz_per_row)
    cols = rng.integers(0, n, size=rows.size)
    v = rng.normal(0.0, 1.0, size=rows.size)
    M = np.zeros((n, n))
    np.add.at(M, (rows, cols), v)
    M = 0.5 * (M + M.T)
    M -= np.diag(np.abs(M).sum(axis=1) + 0.5)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    nzr, nzc = np.nonzero(M)
    np.add.at(rowptr, nzr + 1, 1)
    rowptr = np.cumsum(rowptr)
    colidx = nzc.astype(np.int32)
    vals = M[nzr, nzc]
    gens = []
    starts = np.sort(rng.choice(np.arange(0, n - 8, 8), size=ngen, replace=False))
    for s in starts:
        L = int(rng.integers(1, 8))
        gens.append(Generator(segments_from_ranges([(int(s), int(s) + L)], float(rng.uniform(0.5, 2))),
                              zc=float(rng.uniform(-1, 1)), radius=float(rng.uniform(0.05, 0.3))))
    C = []
    for _ in range(o):
        a = int(rng.integers(0, n - 20))
        C.append(segments_from_ranges([(a, a + int(rng.integers(1, 20)))], float(rng.uniform(0.1, 1))))
    unsafe = np.stack([np.full(o, 0.5), np.full(o, math.inf)], axis=1)
    b = rng.normal(0, 1, size=n) * (rng.uniform(size=n) < 0.1) if affine else None
    ctr = rng.normal(0, 1, size=n) * (rng.uniform(size=n) < 0.05) if center else None
    return Problem("random_symmetric", n, "csr", True, gens, C, unsafe, k=k, dt=dt, steps=steps,
                   b=b, center=ctr, rowptr=rowptr, colidx=colidx, vals=vals, seed=seed)


# ---------------------------------------------------------------------------
# Nonsymmetric 3D convection-diffusion (first-order upwind convection, central
# diffusion, Dirichlet), plus random off-stencil entries
# ---------------------------------------------------------------------------

def conv_diff3d(nx=200, ny=200, nz=250, peclet=5.0, extra_per_row=2, extra_sigma=1e-3, ngen=16,
                gen_len=1000, o=5, k=30, dt=1e-4, steps=1000, seed=3) -> Problem:
    """u' = D lap(u) - v . grad(u) on an nx*ny*nz grid with h = 1/(max dim + 1),
    per-node velocity v ~ U[-1,1]^3, D = h / peclet (cell Peclet number
    max|v_i| h / D = peclet), upwind differences for the convection, and
    `extra_per_row` random off-stencil entries ~ N(0, extra_sigma) per row.
    Generators: indicators of `ngen` disjoint seeded index ranges of length
    `gen_len`, 1.0 +- 0.1; outputs: means over `o` seeded ranges, the first
    two overlapping generator ranges."""
    n = nx * ny * nz
    h = 1.0 / (max(nx, ny, nz) + 1)
    D = h / peclet
    rng = np.random.default_rng(seed)
    vel = rng.uniform(-1.0, 1.0, size=(n, 3))
    idx = np.arange(n, dtype=np.int64)
    iz = idx % nz
    iy = (idx // nz) % ny
    ix = idx // (ny * nz)
    d = D / h**2
    diag = np.full(n, -6.0 * d) - np.abs(vel).sum(axis=1) / h
    cols, vals = [idx], [diag]
    for axis, (coord, m, stride) in enumerate(((ix, nx, ny * nz), (iy, ny, nz), (iz, nz, 1))):
        v = vel[:, axis]
        lo_ok, hi_ok = coord > 0, coord < m - 1
        cols.append(np.where(lo_ok, idx - stride, -1)); vals.append(d + np.maximum(v, 0.0) / h)
        cols.append(np.where(hi_ok, idx + stride, -1)); vals.append(d + np.maximum(-v, 0.0) / h)
    for _ in range(extra_per_row):
        cols.append(rng.integers(0, n, size=n)); vals.append(rng.normal(0.0, extra_sigma, size=n))
    C_ = np.stack(cols, axis=1)
    V_ = np.stack(vals, axis=1)
    rows = np.repeat(idx, C_.shape[1])
    C_ = C_.ravel(); V_ = V_.ravel()
    keep = C_ >= 0
    rows, C_, V_ = rows[keep], C_[keep], V_[keep]
    order = np.lexsort((C_, rows))
    rows, C_, V_ = rows[order], C_[order], V_[order]
    # merge duplicate (row, column) pairs
    first = np.ones(rows.size, dtype=bool)
    first[1:] = (rows[1:] != rows[:-1]) | (C_[1:] != C_[:-1])
    grp = np.cumsum(first) - 1
    vals_m = np.zeros(int(first.sum()))
    np.add.at(vals_m, grp, V_)
    rows_m, cols_m = rows[first], C_[first]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows_m + 1, 1)
    rowptr = np.cumsum(rowptr)
    slots = rng.choice(n // gen_len, size=ngen + o, replace=False) * gen_len
    gens = [Generator(segments_from_ranges([(int(s), int(s) + gen_len)], 1.0), zc=1.0, radius=0.1)
            for s in slots[:ngen]]
    out_starts = list(slots[ngen:ngen + o])
    for q in range(min(2, o)):
        out_starts[q] = min(int(slots[q]) + gen_len // 2, n - gen_len)   # overlaps generator q
    C = [segments_from_ranges([(int(s), int(s) + gen_len)], 1.0 / gen_len) for s in out_starts]
    unsafe = np.stack([np.full(o, 0.5), np.full(o, math.inf)], axis=1)
    return Problem("conv_diff3d", n, "csr", False, gens, C, unsafe, k=k, dt=dt, steps=steps,
                   rowptr=rowptr, colidx=cols_m.astype(np.int32), vals=vals_m, seed=seed,
                   meta={"grid": (nx, ny, nz), "D": D, "h": h},
                   note="nonsymmetric upwind convection-diffusion with random off-stencil entries")


# ---------------------------------------------------------------------------
# Serving stream: seeded verification queries with Poisson arrivals
# ---------------------------------------------------------------------------

# Grid edges of the resident systems: n = m^3 log-spaced from 10^3 to ~10^7.
SERVING_EDGES = (10, 13, 17, 22, 28, 36, 46, 60, 77, 100, 129, 167, 215)
SERVING_DT = {"heat": 0.02, "conv": 1e-4}


def serving_system(family: str, m: int, D=0.01) -> Problem:
    """The system of one resident catalog entry (the generators and outputs
    of a query are attached per query): 3D heat on an m^3 grid as a matrix-
    free stencil (D = 0.01, h = 1/(m+1), Dirichlet), or the convection-
    diffusion matrix of ``conv_diff3d`` on an m^3 grid (seed m)."""
    if family == "heat":
        h = 1.0 / (m + 1)
        c = D / h**2
        coef = (-6.0 * c, c, c, c)
        one = segments_from_ranges([(0, 1)])
        return Problem(f"serve_heat_{m}", m**3, "stencil7", True, [Generator(one, 1.0, 0.1)], [one],
                       np.array([[math.inf, math.inf]]), k=30, dt=SERVING_DT["heat"], steps=100,
                       grid=(m, m, m), coef=coef, seed=m, meta={"m": m})
    p = conv_diff3d(m, m, m, ngen=1, gen_len=1, o=1, k=30, dt=SERVING_DT["conv"], steps=100, seed=m)
    p.name = f"serve_conv_{m}"
    p.meta["m"] = m
    return p


@dataclass
class Query:
    qid: int
    arrival: float           # seconds after the stream starts
    family: str              # "heat" | "conv"
    m: int                   # grid edge of its system (n = m^3)
    gens: list
    C: list
    unsafe: np.ndarray       # (o, 2)
    steps: int
    dt: float
    k: int
    precision: str           # "fp64" | "fp32"
    seed: int

    @property
    def n(self) -> int:
        return self.m ** 3


def serving_query(q: int, arrival: float, seed: int) -> Query:
    """Query q of the stream: heat or convection-diffusion (even odds), size
    n = 10^U[3,7] taken to the nearest resident grid in log scale, 1-8 box
    generators (disjoint seeded index ranges at 1.0 +- 0.1), 1-4 outputs
    (means over seeded ranges, the first one overlapping generator 0),
    100-2000 steps, unsafe when an output reaches theta ~ U[0.05, 1.5],
    FP64 or FP32-basis (even odds), k = 30."""
    rng = np.random.default_rng(seed)
    family = "heat" if rng.uniform() < 0.5 else "conv"
    n_target = 10.0 ** rng.uniform(3.0, 7.0)
    edges = np.array(SERVING_EDGES, dtype=np.float64)
    m = int(SERVING_EDGES[int(np.argmin(np.abs(np.log(edges**3) - math.log(n_target))))])
    n = m**3
    ngen = int(rng.integers(1, 9))
    o = int(rng.integers(1, 5))
    steps = int(rng.integers(100, 2001))
    theta = float(rng.uniform(0.05, 1.5))
    precision = "fp32" if rng.uniform() < 0.5 else "fp64"
    L = max(1, min(1000, n // (4 * (ngen + o))))
    slots = rng.choice(n // L, size=ngen + o, replace=False) * L
    gens = [Generator(segments_from_ranges([(int(s), int(s) + L)], 1.0), zc=1.0, radius=0.1)
            for s in slots[:ngen]]
    out = [int(s) for s in slots[ngen:]]
    out[0] = min(int(slots[0]) + L // 2, n - L)
    C = [segments_from_ranges([(s, s + L)], 1.0 / L) for s in out]
    unsafe = np.array([[theta, math.inf]] * o)
    return Query(q, arrival, family, m, gens, C, unsafe, steps, SERVING_DT[family], 30, precision, seed)


def serving_queries(count: int, rate: float, seed: int = 100):
    """`count` queries with Poisson arrivals at `rate` per second (seeded
    exponential gaps); query q draws its own parameters from seed + q."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    return [serving_query(q, float(arrivals[q]), seed + q) for q in range(count)]


def query_problem(system: Problem, query: Query) -> Problem:
    """The whole Problem of one query (its system with its generators,
    outputs, unsafe set and time grid), e.g. for the oracle."""
    p = Problem(f"{system.name}_q{query.qid}", system.n, system.kind, system.symmetric, query.gens, query.C,
                query.unsafe, k=query.k, dt=query.dt, steps=query.steps, rowptr=system.rowptr,
                colidx=system.colidx, vals=system.vals, grid=system.grid, coef=system.coef, seed=query.seed)
    return p
