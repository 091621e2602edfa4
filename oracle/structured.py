"""Kronecker operator applied to structured (CP, Tucker, TT) magnetizations.

TEST INFRASTRUCTURE ONLY (see the package header).

Paper: Sec. 3.4, Eqs. (kron_eval), (kron_eval_cp), (kron_eval_tuck) (the
U_k^(q1) V^(3) in the printed formulas is read as U_k^(q3) V^(3)); Sec. 4.1
Lemmas DFT_cp / DFT_tucker (the structured DFT acts column-wise on factors);
App. C, Eq. (tt_3d_2) (a 3D TT is the Tucker2 form [[G2; G1, id, G3^T]]).

Every factor-matrix product here is a dense Toeplitz matrix (Sec. 4.2) times a
column, in float64; nothing is transformed.  The results are uncompressed sums
of terms (block-CP, Sec. 2.2): per output o in (phi, h_x, h_y, h_z), input
component q and node k, one CP/Tucker/TT term whose axis-d factor is
T_{d, type(o, q, d), k} times the input's axis-d factor.

Column numbering (shared convention of the library's result tables):
for axis d, input component q, "derivative slot" s and node k, the column of
input factor column l is
    col_d(q, s, k, l) = ((q * 2 + s) * M + k) * r_d + l,
where s = 1 exactly when the output is the field component h_d (the factor in
axis d is the differentiated one: P~ if d == q else Q~), s = 0 otherwise
(X~ if d == q else E~).  For TT inputs axis y has r_d = r1 * r2 fibre columns
numbered l = a * r2 + b for G2[a, :, b].
"""
from __future__ import annotations

import numpy as np

from . import sinc

OUTPUTS = ("phi", "hx", "hy", "hz")


def slot(o: int, d: int) -> int:
    """s = 1 iff output o (0 = phi, 1..3 = h_x..h_z) is the field along d."""
    return 1 if o == d + 1 else 0


def type_of(q: int, d: int, s: int) -> int:
    if d == q:
        return sinc.TYPE_P if s else sinc.TYPE_X
    return sinc.TYPE_Q if s else sinc.TYPE_E


def _columns(F_d, q, d, cols_in, M):
    """Output columns for axis d, component q: array [2][M][r][n_d]."""
    r = cols_in.shape[1]
    out = np.empty((2, M, r, cols_in.shape[0]))
    for s in range(2):
        t = type_of(q, d, s)
        for k in range(M):
            out[s, k] = (sinc.toeplitz(F_d[t, k]) @ cols_in).T
    return out


def term_table(M: int, r: int):
    """CP term table: int array [4][3*M*r][3] of column indices per axis,
    term index (q * M + k) * r + l."""
    tab = np.empty((4, 3 * M * r, 3), dtype=np.int32)
    for o in range(4):
        for q in range(3):
            for k in range(M):
                for l in range(r):
                    t = (q * M + k) * r + l
                    for d in range(3):
                        tab[o, t, d] = ((q * 2 + slot(o, d)) * M + k) * r + l
    return tab


def block_table(M: int, ranks):
    """Tucker/TT block table: int array [4][3*M][3] of the first column per
    axis of block (q, k) (block index q * M + k); its columns are contiguous."""
    tab = np.empty((4, 3 * M, 3), dtype=np.int32)
    for o in range(4):
        for q in range(3):
            for k in range(M):
                for d in range(3):
                    tab[o, q * M + k, d] = ((q * 2 + slot(o, d)) * M + k) * ranks[d]
    return tab


def cp_apply(cp, n, h, tau, alpha):
    """Returns (cols[d] arrays [3*2*M*r][n_d], weights lam[q] per term, table)."""
    M = len(tau)
    F = [sinc.scaled_factors(n[d], h[d], tau, alpha) for d in range(3)]
    r = cp.lam[0].size
    cols = []
    for d in range(3):
        per_q = [_columns(F[d], q, d, np.asarray(cp.U[q][d], dtype=np.float64), M) for q in range(3)]
        cols.append(np.stack(per_q).reshape(3 * 2 * M * r, n[d]))
    return cols, term_table(M, r)


def cp_densify(cols, table, lam, M, r, n):
    """Dense [4][nz][ny][nx] from CP result columns (term weight lam[q][l])."""
    nx, ny, nz = n
    out = np.zeros((4, nz, ny, nx))
    for o in range(4):
        for q in range(3):
            for k in range(M):
                for l in range(r):
                    t = (q * M + k) * r + l
                    cx, cy, cz = table[o, t]
                    out[o] += lam[q][l] * np.einsum("z,y,x->zyx", cols[2][cz], cols[1][cy], cols[0][cx])
    return out


def cp_to_full(cp, n):
    """Dense m[3][nz][ny][nx] of a CP magnetization (Eq. (CP))."""
    return np.stack([np.einsum("r,xr,yr,zr->zyx", cp.lam[q], cp.U[q][0], cp.U[q][1], cp.U[q][2])
                     for q in range(3)])


def tucker_apply(tk, n, h, tau, alpha):
    """Returns (cols[d] arrays [3*2*M*r_d][n_d], table)."""
    M = len(tau)
    F = [sinc.scaled_factors(n[d], h[d], tau, alpha) for d in range(3)]
    ranks = tk.core[0].shape
    cols = []
    for d in range(3):
        per_q = [_columns(F[d], q, d, np.asarray(tk.U[q][d], dtype=np.float64), M) for q in range(3)]
        cols.append(np.stack(per_q).reshape(3 * 2 * M * ranks[d], n[d]))
    return cols, block_table(M, ranks)


def tucker_densify(cols, table, core, M, n):
    """Dense [4][nz][ny][nx]: sum over blocks of [[C^q; Ux, Uy, Uz]] (Eq. (tucker_rep))."""
    nx, ny, nz = n
    ranks = core[0].shape
    out = np.zeros((4, nz, ny, nx))
    for o in range(4):
        for q in range(3):
            for k in range(M):
                c0 = table[o, q * M + k]
                Ux = cols[0][c0[0]:c0[0] + ranks[0]]
                Uy = cols[1][c0[1]:c0[1] + ranks[1]]
                Uz = cols[2][c0[2]:c0[2] + ranks[2]]
                out[o] += np.einsum("abc,ax,by,cz->zyx", core[q], Ux, Uy, Uz)
    return out


def tucker_to_full(tk, n):
    return np.stack([np.einsum("abc,xa,yb,zc->zyx", tk.core[q], tk.U[q][0], tk.U[q][1], tk.U[q][2])
                     for q in range(3)])


def tt_apply(tt, n, h, tau, alpha):
    """TT input (App. C): axis x acts on G1's columns, axis y on the r1*r2
    fibres G2[a, :, b], axis z on the rows of G3.  Returns (cols, table)."""
    M = len(tau)
    F = [sinc.scaled_factors(n[d], h[d], tau, alpha) for d in range(3)]
    r1 = tt.G1[0].shape[1]
    r2 = tt.G3[0].shape[0]
    ranks = (r1, r1 * r2, r2)
    cols = [[], [], []]
    for q in range(3):
        inx = np.asarray(tt.G1[q], dtype=np.float64)                       # (nx, r1)
        iny = np.asarray(tt.G2[q], dtype=np.float64).transpose(1, 0, 2).reshape(n[1], r1 * r2)
        inz = np.asarray(tt.G3[q], dtype=np.float64).T                     # (nz, r2)
        for d, cin in enumerate((inx, iny, inz)):
            cols[d].append(_columns(F[d], q, d, cin, M))
    cols = [np.stack(cols[d]).reshape(3 * 2 * M * ranks[d], n[d]) for d in range(3)]
    return cols, block_table(M, ranks)


def tt_densify(cols, table, M, n, r1, r2):
    nx, ny, nz = n
    out = np.zeros((4, nz, ny, nx))
    for o in range(4):
        for q in range(3):
            for k in range(M):
                c0 = table[o, q * M + k]
                G1 = cols[0][c0[0]:c0[0] + r1].T                              # (nx, r1)
                G2 = cols[1][c0[1]:c0[1] + r1 * r2].reshape(r1, r2, ny)       # [a][b][y]
                G3 = cols[2][c0[2]:c0[2] + r2]                                # (r2, nz)
                out[o] += np.einsum("xa,aby,bz->zyx", G1, G2, G3)
    return out


def tt_to_full(tt, n):
    return np.stack([np.einsum("xa,ayb,bz->zyx", tt.G1[q], tt.G2[q], tt.G3[q]) for q in range(3)])
