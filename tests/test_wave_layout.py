"""Lane-level model of the wavefront translation kernel's index mapping (host
only).  The 16x16x4 matrix-core instruction takes A[l % 16][l / 16] and
B[l / 16][l % 16] from lane l and returns register q of lane l as
D[4q + l/16][l % 16] (FP64) or D[4(l/16) + q][l % 16] (FP32).  The model
feeds lanes exactly as the kernel does: real inner index 16 g + 4 k4 + t for
lane group k4 at step (g, t), A rows permuted by rho so that register q of
lane group k4 holds real row 4 k4 + q, the low-rank T = V X handed to the
second product straight from the result registers, and two complex outputs
stored per lane.  It must reproduce the complex products M X and U (V X) for
dense and low-rank operators, both result layouts, ragged row, column, rank
and pair counts, and store nothing past the chunk's pairs."""
import numpy as np
import pytest

LANE = np.arange(64)
I16, K4 = LANE & 15, LANE >> 4


def mma(a, b, acc, f64):
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    A[I16, K4] = a
    B[K4, I16] = b
    D = A @ B
    q = np.arange(4)[None, :]
    rows = 4 * q + K4[:, None] if f64 else 4 * K4[:, None] + q
    return acc + D[rows, I16[:, None]]


def rho(m, f64):
    return 4 * (m & 3) + (m >> 2) if f64 else m


def a_group(M, nrow, ncol, I, j0):
    """Four A values per lane: row I (real) against complex columns j0, j0 + 1."""
    i, c = I >> 1, I & 1
    out = np.zeros((64, 4))
    for l in range(64):
        m0 = M[i[l], j0[l]] if (i[l] < nrow and j0[l] < ncol) else 0j
        m1 = M[i[l], j0[l] + 1] if (i[l] < nrow and j0[l] + 1 < ncol) else 0j
        if c[l]:
            out[l] = (m0.imag, m0.real, m1.imag, m1.real)
        else:
            out[l] = (m0.real, -m0.imag, m1.real, -m1.imag)
    return out


def b_group(X, ncol, j0, pok):
    out = np.zeros((64, 4))
    for l in range(64):
        p = I16[l]
        x0 = X[j0[l], p] if (pok[l] and j0[l] < ncol) else 0j
        x1 = X[j0[l] + 1, p] if (pok[l] and j0[l] + 1 < ncol) else 0j
        out[l] = (x0.real, x0.imag, x1.real, x1.imag)
    return out


def chunk(M, U, V, X, npairs, s, cols, r, f64):
    Y = np.full((s, 16), np.nan + 0j)
    pok = I16 < npairs

    def store(rt, acc):
        for l in range(64):
            if not pok[l]:
                continue
            m0 = 8 * rt + 2 * K4[l]
            if m0 < s:
                Y[m0, I16[l]] = acc[l, 0] + 1j * acc[l, 1]
            if m0 + 1 < s:
                Y[m0 + 1, I16[l]] = acc[l, 2] + 1j * acc[l, 3]

    n_rt, G, rw = (2 * s + 15) >> 4, (2 * cols + 15) >> 4, rho(I16, f64)
    if r < 0:
        for rt in range(n_rt):
            acc = np.zeros((64, 4))
            for g in range(G):
                a = a_group(M, s, cols, 16 * rt + rw, 8 * g + 2 * K4)
                b = b_group(X, cols, 8 * g + 2 * K4, pok)
                for t in range(4):
                    acc = mma(a[:, t], b[:, t], acc, f64)
            store(rt, acc)
        return Y
    RT = max(1, (2 * r + 15) >> 4)
    T = [np.zeros((64, 4)) for _ in range(RT)]
    for g in range(G):
        b = b_group(X, cols, 8 * g + 2 * K4, pok)
        for q in range(RT):
            a = a_group(V, r, cols, 16 * q + rw, 8 * g + 2 * K4)
            for t in range(4):
                T[q] = mma(a[:, t], b[:, t], T[q], f64)
    for rt in range(n_rt):
        acc = np.zeros((64, 4))
        for q in range(RT):
            a = a_group(U, s, r, 16 * rt + rw, 8 * q + 2 * K4)
            for u in range(4):
                acc = mma(a[:, u], T[q][:, u], acc, f64)
        store(rt, acc)
    return Y


@pytest.mark.parametrize("f64", [True, False])
@pytest.mark.parametrize("s,cols,r,npairs", [(9, 9, -1, 16), (11, 7, 3, 13), (5, 13, 9, 5), (12, 10, 0, 16),
                                             (3, 18, -1, 1)])
def test_wavefront_chunk_index_mapping(f64, s, cols, r, npairs):
    rng = np.random.default_rng(s * 100 + cols)

    def cr(*sh):
        return rng.standard_normal(sh) + 1j * rng.standard_normal(sh)

    X = cr(cols, 16)
    if r < 0:
        M, U, V = cr(s, cols), None, None
        ref = M @ X
    else:
        M, U, V = None, cr(s, max(r, 1))[:, :r], cr(max(r, 1), cols)[:r]
        ref = U @ (V @ X)
    Y = chunk(M, U, V, X, npairs, s, cols, r, f64)
    assert np.all(np.isnan(Y[:, npairs:])), "stored past the chunk's pairs"
    assert np.abs(Y[:, :npairs] - ref[:, :npairs]).max() <= 1e-12 * max(1.0, np.abs(ref).max())
