"""Plain FP64 reference of the EPIC imaging path.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports or calls this
module; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It is deliberately slow and literal: every step is the definition
written out in float64/complex128 with NumPy, with no blocking, fusion or
reordering beyond what the definition states.

What it computes (paper: Sec. 2, Eq. 1 and Eq. 2):

* Eq. 1, inner sum: each calibrated voltage E_e^p is spread onto a regular
  aperture grid r_j with the conjugate of its element's gridding kernel,
  G^p[j] = sum_e W_e*(r_j - r_e) E_e^p.  The default kernel is diagonal in
  polarisation (the same kernel for both feeds); the ``*_jones`` functions
  take the full form of Eq. 1, G^alpha[j] = sum_e sum_p W_e^{alpha p}*(r_j -
  r_e) E_e^p, with four complex kernels per element.
* Eq. 1, outer sum: a 2D Fourier sum with the positive exponent,
  E^p[k] = sum_j dA_j exp(+2 pi i s_k . r_j / lambda) G^p[j], written on
  centred integer indices as exp(+2 pi i (k - N/2).(j - N/2) / N), with the
  cell area dA_j taken as 1.
* Eq. 2: pixelwise outer product of polarisations, E^a conj(E^b), summed
  over the integration; XX, YY and XY = Ex conj(Ey) are kept.
* Autocorrelation removal: the e = e' terms of the squared sum.  They are
  sum_a S_a^{pq} |B_a[k]|^2 with S_a^{pq} = sum_t E_a^p conj(E_a^q) and
  B_a the image of element a's kernel footprint alone.
* The FX route: form every pairwise visibility V_ab = sum_t E_a conj(E_b)
  explicitly, grid it at the footprint displacements with the correlated
  kernel conj(W_a(j)) W_b(j'), and Fourier transform.  Expanding |sum|^2 in
  Eq. 1/2 shows it equals the EPIC image exactly (all pairs), and the
  autocorrelation-removed EPIC image equals FX over a != b.

Readings where the paper is silent (grid geometry, kernel shape, voltage
packing) are the ones listed in the design notes: cell = cell_lambda *
lambda, grid index of an element x = pos / cell + N/2, support start
j0 = floor(x - K/2 + 1), a Gaussian kernel of width sigma cells truncated to
K x K and normalised to unit sum, 4+4-bit two's-complement voltages with the
real part in the high nibble.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0

__all__ = [
    "C_LIGHT", "decode_int4", "grid_geometry", "gaussian_kernel",
    "support_inside", "grid", "centred_dft_matrix", "sky", "n_products",
    "accumulate", "antenna_autos", "antenna_beams", "auto_term", "auto_term_by_element",
    "readout",
    "fx_image", "channel_reference", "decode_int8", "decode_voltages",
    "pseudo_stokes", "grid_jones", "antenna_beams_jones", "auto_term_jones",
    "fx_image_jones",
]


# --------------------------------------------------------------------------
# Voltages
# --------------------------------------------------------------------------
def decode_int8(v) -> np.ndarray:
    """8+8-bit samples ``int8 [..., 2]`` (real, imaginary) -> complex integer
    (the digitisation of the paper's synthetic test, Sec. 4)."""
    v = np.asarray(v, dtype=np.int8).astype(np.float64)
    return v[..., 0] + 1j * v[..., 1]


def decode_voltages(v) -> np.ndarray:
    """Either format: packed 4+4-bit bytes, or int8 (re, im) pairs in a
    trailing axis of length 2."""
    v = np.asarray(v)
    if v.dtype == np.int8 and v.shape[-1] == 2:
        return decode_int8(v)
    return decode_int4(v)


def decode_int4(b) -> np.ndarray:
    """4+4-bit packed byte -> complex integer (Sec. 4 digitised voltages).

    High nibble = real, low nibble = imaginary, two's complement (so 0x8
    decodes to -8).
    """
    b = np.asarray(b, dtype=np.uint8).astype(np.int16)
    hi = b >> 4
    lo = b & 0xF
    hi = np.where(hi >= 8, hi - 16, hi)
    lo = np.where(lo >= 8, lo - 16, lo)
    return hi.astype(np.float64) + 1j * lo.astype(np.float64)


# --------------------------------------------------------------------------
# Grid geometry and kernel (Eq. 1 inner sum; Sec. 4 grid spacing)
# --------------------------------------------------------------------------
def grid_geometry(pos, freq_hz, n, cell_lambda=0.5, k=3):
    """Element positions in grid units and the first cell of each support.

    The grid point j sits at (j - N/2) * cell metres, with
    cell = cell_lambda * lambda.  Returns ``x`` (float64 [A][2], (east,
    north) in cells) and ``j0`` (int64 [A][2]) such that the K x K support
    of element a covers cells j0 .. j0+K-1 on each axis.
    """
    pos = np.asarray(pos, dtype=np.float64)
    lam = C_LIGHT / float(freq_hz)
    cell = cell_lambda * lam
    x = pos / cell + n / 2.0
    j0 = np.floor(x - k / 2.0 + 1.0).astype(np.int64)
    return x, j0


def gaussian_kernel(x, j0, k=3, sigma=0.5):
    """Real, unit-sum Gaussian kernel sampled on each element's support.

    Returns ``w`` float64 [A][K][K] indexed [a][dy][dx], the weight on cell
    (j0y + dy, j0x + dx).
    """
    x = np.asarray(x, dtype=np.float64)
    A = x.shape[0]
    w = np.zeros((A, k, k))
    for a in range(A):
        for dy in range(k):
            for dx in range(k):
                ex = j0[a, 0] + dx - x[a, 0]
                ey = j0[a, 1] + dy - x[a, 1]
                w[a, dy, dx] = np.exp(-(ex * ex + ey * ey) / (2.0 * sigma * sigma))
        w[a] /= w[a].sum()
    return w


def support_inside(j0, k, n, aperture_n=0) -> bool:
    """True when every support lies inside the gridded region.

    The gridded region is the central ``aperture_n`` cells of the N-grid
    (all of it when ``aperture_n`` is 0).
    """
    m = n if aperture_n in (0, None) else aperture_n
    lo = (n - m) // 2
    hi = lo + m - 1
    return bool(np.all(j0 >= lo) and np.all(j0 + k - 1 <= hi))


def grid(E, j0, w, n) -> np.ndarray:
    """Eq. 1 inner sum: G[jy][jx] = sum_a conj(w_a(j)) E_a.

    ``E`` is complex [..., A]; returns complex128 [..., N, N].
    """
    E = np.asarray(E, dtype=np.complex128)
    A = E.shape[-1]
    k = w.shape[-1]
    G = np.zeros(E.shape[:-1] + (n, n), dtype=np.complex128)
    wc = np.conj(w)
    for a in range(A):
        for dy in range(k):
            for dx in range(k):
                G[..., j0[a, 1] + dy, j0[a, 0] + dx] += wc[a, dy, dx] * E[..., a]
    return G


def grid_jones(E, j0, wj, n) -> np.ndarray:
    """Eq. 1 inner sum with polarisation mixing:
    G^alpha[j] = sum_a sum_p conj(W_a^{alpha p}(j)) E_a^p.

    ``E`` is complex [..., 2, A] (feed p, element); ``wj`` is complex
    [A][2][2][K][K] indexed (element, alpha, p, dy, dx).  Returns complex128
    [..., 2, N, N] (output polarisation alpha).
    """
    E = np.asarray(E, dtype=np.complex128)
    A = E.shape[-1]
    k = wj.shape[-1]
    G = np.zeros(E.shape[:-2] + (2, n, n), dtype=np.complex128)
    wc = np.conj(wj)
    for a in range(A):
        for al in range(2):
            for p in range(2):
                for dy in range(k):
                    for dx in range(k):
                        G[..., al, j0[a, 1] + dy, j0[a, 0] + dx] += wc[a, al, p, dy, dx] * E[..., p, a]
    return G


def centred_dft_matrix(n) -> np.ndarray:
    """F[k][j] = exp(+2 pi i (k - N/2)(j - N/2) / N) (Eq. 1 outer sum).

    The exponent is reduced modulo N in integer arithmetic before the
    exponential so every entry is accurate to float64 rounding.
    """
    idx = np.arange(n, dtype=np.int64) - n // 2
    p = np.mod(np.outer(idx, idx), n).astype(np.float64)
    return np.exp(2j * np.pi * p / n)


def sky(G) -> np.ndarray:
    """Eq. 1 outer sum on a grid G[..., jy, jx]: returns E[..., ky, kx].

    Separable direct DFT: E = F G F^T with F from ``centred_dft_matrix``.
    """
    G = np.asarray(G, dtype=np.complex128)
    F = centred_dft_matrix(G.shape[-1])
    return F @ G @ F.T


# --------------------------------------------------------------------------
# Eq. 2: polarisation products and the time sum
# --------------------------------------------------------------------------
def n_products(n_pol: int) -> int:
    """XX only for one feed; XX, YY, Re XY, Im XY for two."""
    return 1 if n_pol == 1 else 4


def accumulate(Esky) -> np.ndarray:
    """Eq. 2 summed over time from sky images ``Esky`` [T][P][N][N].

    Returns float64 [n_prod][N][N]: XX = sum |Ex|^2, YY = sum |Ey|^2 and
    XY = sum Ex conj(Ey) split into real and imaginary planes.
    """
    Esky = np.asarray(Esky)
    P = Esky.shape[1]
    ex = Esky[:, 0]
    xx = np.sum(np.abs(ex) ** 2, axis=0)
    if P == 1:
        return xx[None]
    ey = Esky[:, 1]
    yy = np.sum(np.abs(ey) ** 2, axis=0)
    xy = np.sum(ex * np.conj(ey), axis=0)
    return np.stack([xx, yy, xy.real, xy.imag])


def antenna_autos(E) -> np.ndarray:
    """Per-element time sums S_a^{pq} = sum_t E_a^p conj(E_a^q).

    ``E`` is complex [T][P][A]; returns float64 [A][n_prod] in the same
    product order as ``accumulate`` (values are exact integers for int4
    inputs).
    """
    E = np.asarray(E)
    P = E.shape[1]
    # |E|^2 as re^2 + im^2: exact for integer samples (abs() then squaring
    # rounds through a square root)
    xx = np.sum(E[:, 0].real ** 2 + E[:, 0].imag ** 2, axis=0)
    if P == 1:
        return xx[:, None]
    yy = np.sum(E[:, 1].real ** 2 + E[:, 1].imag ** 2, axis=0)
    xy = np.sum(E[:, 0] * np.conj(E[:, 1]), axis=0)
    return np.stack([xx, yy, xy.real, xy.imag], axis=1)


def antenna_beams(j0, w, n) -> np.ndarray:
    """B_a[k]: the Eq. 1 image of element a's kernel footprint alone.

    B_a[ky][kx] = sum_{dy,dx} conj(w_a[dy][dx]) F[ky][j0y+dy] F[kx][j0x+dx].
    Returns complex128 [A][N][N].
    """
    F = centred_dft_matrix(n)
    A, k = w.shape[0], w.shape[-1]
    B = np.zeros((A, n, n), dtype=np.complex128)
    wc = np.conj(w)
    for a in range(A):
        Fy = F[:, j0[a, 1]:j0[a, 1] + k]          # [N][K]
        Fx = F[:, j0[a, 0]:j0[a, 0] + k]
        B[a] = Fy @ wc[a] @ Fx.T
    return B


def auto_term(S, B) -> np.ndarray:
    """sum_a S_a^{pq} |B_a[k]|^2 for each stored product.

    The same kernel serves both feeds, so every product's self term is the
    element's power pattern weighted by its own auto sum.
    """
    P2 = np.abs(B) ** 2                              # [A][N][N]
    return np.einsum("ap,ayx->pyx", np.asarray(S, dtype=np.float64), P2)


def auto_term_by_element(S, j0, w, n) -> np.ndarray:
    """The same sum as ``auto_term(S, antenna_beams(j0, w, n))``, adding one
    element's power pattern at a time so memory stays O(N^2)."""
    F = centred_dft_matrix(n)
    S = np.asarray(S, dtype=np.float64)
    k = w.shape[-1]
    wc = np.conj(w)
    out = np.zeros((S.shape[1], n, n))
    for a in range(S.shape[0]):
        Fy = F[:, j0[a, 1]:j0[a, 1] + k]
        Fx = F[:, j0[a, 0]:j0[a, 0] + k]
        p2 = np.abs(Fy @ wc[a] @ Fx.T) ** 2
        out += S[a][:, None, None] * p2
    return out


def antenna_beams_jones(j0, wj, n) -> np.ndarray:
    """B_a^{alpha p}[k]: the Eq. 1 image of element a's footprint for feed p
    into output polarisation alpha.  Returns complex128 [A][2][2][N][N]."""
    F = centred_dft_matrix(n)
    A, k = wj.shape[0], wj.shape[-1]
    B = np.zeros((A, 2, 2, n, n), dtype=np.complex128)
    wc = np.conj(wj)
    for a in range(A):
        Fy = F[:, j0[a, 1]:j0[a, 1] + k]
        Fx = F[:, j0[a, 0]:j0[a, 0] + k]
        for al in range(2):
            for p in range(2):
                B[a, al, p] = Fy @ wc[a, al, p] @ Fx.T
    return B


def auto_term_jones(S, Bj) -> np.ndarray:
    """Self terms with polarisation mixing.  Element a alone contributes
    E^alpha = sum_p B_a^{alpha p} E_a^p to every pixel, so its share of
    sum_t E^alpha conj(E^beta) is sum_{p,q} S_a^{pq} B_a^{alpha p}
    conj(B_a^{beta q}), with S_a^{yx} = conj(S_a^{xy}).  ``S`` is [A][4]
    (XX, YY, Re XY, Im XY) as from ``antenna_autos``; returns float64
    [4][N][N] in the same product order."""
    S = np.asarray(S, dtype=np.float64)
    sxy = S[:, 2] + 1j * S[:, 3]
    Sm = np.empty((S.shape[0], 2, 2), dtype=np.complex128)
    Sm[:, 0, 0] = S[:, 0]
    Sm[:, 1, 1] = S[:, 1]
    Sm[:, 0, 1] = sxy
    Sm[:, 1, 0] = np.conj(sxy)

    def one(al, be):
        out = np.zeros(Bj.shape[-2:], dtype=np.complex128)
        for p in range(2):
            for q in range(2):
                out += np.einsum("a,ayx->yx", Sm[:, p, q],
                                 Bj[:, al, p] * np.conj(Bj[:, be, q]))
        return out

    xx, yy, xy = one(0, 0), one(1, 1), one(0, 1)
    return np.stack([xx.real, yy.real, xy.real, xy.imag])


def readout(acc, auto=None, count=1, normalise=True) -> np.ndarray:
    """(acc - auto) / count: Eq. 2's average with the self terms removed."""
    out = np.array(acc, dtype=np.float64, copy=True)
    if auto is not None:
        out -= auto
    if normalise:
        out /= float(count)
    return out


# --------------------------------------------------------------------------
# FX route (pairwise visibilities) -- the brute-force equivalence check
# --------------------------------------------------------------------------
def pseudo_stokes(img) -> np.ndarray:
    """Pseudo-Stokes planes of a two-feed image set [XX, YY, Re XY, Im XY]
    (linear feeds, XY = Ex conj(Ey)): I = XX + YY, Q = XX - YY,
    U = XY + YX = 2 Re XY, V = i (XY - YX) = -2 Im XY."""
    img = np.asarray(img, dtype=np.float64)
    xx, yy, xr, xi = img
    return np.stack([xx + yy, xx - yy, 2 * xr, -2 * xi])


def fx_image(E, j0, w, n, include_auto=True) -> np.ndarray:
    """Image from explicit visibilities gridded with the correlated kernel.

    V_ab^{pq} = sum_t E_a^p conj(E_b^q) is placed at displacement
    d = ja - jb with weight conj(w_a(ja)) w_b(jb) for every pair of support
    cells, on a (2N-1)^2 displacement grid, then
    I[k] = sum_d D[d] exp(+2 pi i (k - N/2).d / N).
    Returns float64 [n_prod][N][N] like ``accumulate``.
    """
    E = np.asarray(E, dtype=np.complex128)
    T, P, A = E.shape
    k = w.shape[-1]
    wc = np.conj(w)
    m = 2 * n - 1
    # displacement transform Q[k][d], d index = displacement + (n - 1)
    kk = np.arange(n) - n // 2
    dd = np.arange(m) - (n - 1)
    Q = np.exp(2j * np.pi * np.mod(np.outer(kk, dd), n) / n)

    def one(p, q):
        V = E[:, p, :].T @ np.conj(E[:, q, :])        # [A][A], V[a][b]
        D = np.zeros((m, m), dtype=np.complex128)
        for a in range(A):
            for b in range(A):
                if a == b and not include_auto:
                    continue
                for ay in range(k):
                    for ax in range(k):
                        ca = wc[a, ay, ax] * V[a, b]
                        for by in range(k):
                            for bx in range(k):
                                dy = (j0[a, 1] + ay) - (j0[b, 1] + by) + n - 1
                                dx = (j0[a, 0] + ax) - (j0[b, 0] + bx) + n - 1
                                D[dy, dx] += ca * w[b, by, bx]
        return Q @ D @ Q.T

    xx = one(0, 0)
    if P == 1:
        return np.stack([xx.real])
    yy = one(1, 1)
    xy = one(0, 1)
    return np.stack([xx.real, yy.real, xy.real, xy.imag])


def fx_image_jones(E, j0, wj, n, include_auto=True) -> np.ndarray:
    """FX route with polarisation mixing: every pairwise visibility
    V_ab^{pq} = sum_t E_a^p conj(E_b^q) is placed at displacement
    d = ja - jb with weight conj(W_a^{alpha p}(ja)) W_b^{beta q}(jb), summed
    over p and q for output product alpha beta, then Fourier transformed as
    in ``fx_image``.  Returns float64 [4][N][N] (XX, YY, Re XY, Im XY)."""
    E = np.asarray(E, dtype=np.complex128)
    T, P, A = E.shape
    k = wj.shape[-1]
    wc = np.conj(wj)
    m = 2 * n - 1
    kk = np.arange(n) - n // 2
    dd = np.arange(m) - (n - 1)
    Q = np.exp(2j * np.pi * np.mod(np.outer(kk, dd), n) / n)
    V = np.einsum("tpa,tqb->pqab", E, np.conj(E))     # V[p][q][a][b]

    def one(al, be):
        D = np.zeros((m, m), dtype=np.complex128)
        for a in range(A):
            for b in range(A):
                if a == b and not include_auto:
                    continue
                for p in range(2):
                    for q in range(2):
                        v = V[p, q, a, b]
                        for ay in range(k):
                            for ax in range(k):
                                ca = wc[a, al, p, ay, ax] * v
                                for by in range(k):
                                    for bx in range(k):
                                        dy = (j0[a, 1] + ay) - (j0[b, 1] + by) + n - 1
                                        dx = (j0[a, 0] + ax) - (j0[b, 0] + bx) + n - 1
                                        D[dy, dx] += ca * wj[b, be, q, by, bx]
        return Q @ D @ Q.T

    xx, yy, xy = one(0, 0), one(1, 1), one(0, 1)
    return np.stack([xx.real, yy.real, xy.real, xy.imag])


# --------------------------------------------------------------------------
# Whole path for one channel / a whole block
# --------------------------------------------------------------------------
def channel_reference(volt_c, pos, freq_hz, n, *, cell_lambda=0.5, k=3,
                      sigma=0.5, kernel=None, aperture_n=0,
                      want_images=False, want_auto=True, jones=None):
    """Reference for one channel of voltages ``uint8 [T][P][A]`` (4+4 bit) or
    ``int8 [T][P][A][2]`` (8+8 bit).

    ``kernel`` optionally replaces the Gaussian with explicit complex weights
    [A][K][K] (the weight W_a on each support cell).  ``jones`` (two feeds
    only) instead gives the four kernels W_a^{alpha p} per element, complex
    [A][2][2][K][K], and the grids mix the feeds as in Eq. 1.  Returns a dict with
    ``acc`` (float64 [n_prod][N][N]), ``autos`` ([A][n_prod]), ``auto``
    (the self term, same shape as acc), ``j0``, ``w`` and, on request, the
    per-sample grids and sky images.  ``want_auto=False`` leaves ``auto``
    as None (its cost grows as A N^2).
    """
    E = decode_voltages(volt_c)                      # [T][P][A]
    x, j0 = grid_geometry(pos, freq_hz, n, cell_lambda, k)
    if not support_inside(j0, k, n, aperture_n):
        raise ValueError("an element's kernel support leaves the gridded region")
    if jones is not None:
        if E.shape[1] != 2:
            raise ValueError("Jones kernels need two feeds")
        w = np.asarray(jones, dtype=np.complex128)
        G = grid_jones(E, j0, w, n)                  # [T][2][N][N]
    else:
        w = gaussian_kernel(x, j0, k, sigma) if kernel is None else \
            np.asarray(kernel, dtype=np.complex128)
        G = grid(E, j0, w, n)                        # [T][P][N][N]
    Es = sky(G)
    acc = accumulate(Es)
    S = antenna_autos(E)
    if not want_auto:
        auto = None
    elif jones is not None:
        # linear in the elements: sum over blocks of elements keeps memory low
        auto = np.zeros_like(acc)
        step = max(1, (1 << 22) // (4 * n * n))
        for a0 in range(0, len(j0), step):
            sl = slice(a0, a0 + step)
            auto += auto_term_jones(S[sl], antenna_beams_jones(j0[sl], w[sl], n))
    elif len(j0) * n * n <= (1 << 24):
        auto = auto_term(S, antenna_beams(j0, w, n))
    else:
        auto = auto_term_by_element(S, j0, w, n)
    out = dict(acc=acc, autos=S, auto=auto, j0=j0, w=w, x=x, count=E.shape[0])
    if want_images:
        out["grid"] = G
        out["sky"] = Es
    return out
