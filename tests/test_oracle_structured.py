"""Pins of the structured-input references (oracle.structured) and of the
bfloat16 split emulation (oracle.bf16)."""
import numpy as np
import pytest
import torch

from oracle import apply, bf16, exact, sinc, structured
from paper_1212_3509_amd import inputs

N_SMALL = (9, 8, 7)
H_SMALL = (1 / 9, 1 / 9, 1 / 9)


def _rule(M=6):
    _t, tau, alpha = sinc.sinc_nodes(M)
    return tau, alpha


def test_cp_apply_equals_full_apply():
    """Eq. (kron_eval_cp): applying the Kronecker operator factor-wise to a CP
    tensor gives the same tensor as the full-format apply of its densification."""
    tau, alpha = _rule()
    cp = inputs.cp_input(N_SMALL, rank=3, seed=1)
    cols, tab = structured.cp_apply(cp, N_SMALL, H_SMALL, tau, alpha)
    dense = structured.cp_densify(cols, tab, cp.lam, len(tau), 3, N_SMALL)
    phi, hf = apply.kron_apply_dense(structured.cp_to_full(cp, N_SMALL), H_SMALL, tau, alpha)
    assert apply.rel_l2(dense[0], phi) < 1e-13
    assert apply.rel_l2(dense[1:], hf) < 1e-13


def test_tucker_apply_equals_full_apply():
    """Eq. (kron_eval_tuck)."""
    tau, alpha = _rule()
    tk = inputs.tucker_input(N_SMALL, ranks=(2, 3, 2), seed=1)
    cols, tab = structured.tucker_apply(tk, N_SMALL, H_SMALL, tau, alpha)
    dense = structured.tucker_densify(cols, tab, tk.core, len(tau), N_SMALL)
    phi, hf = apply.kron_apply_dense(structured.tucker_to_full(tk, N_SMALL), H_SMALL, tau, alpha)
    assert apply.rel_l2(dense[0], phi) < 1e-13
    assert apply.rel_l2(dense[1:], hf) < 1e-13


def test_tt_apply_equals_full_apply():
    """App. C, Eq. (tt_3d_2): a 3D TT is a Tucker2 tensor, so the operator acts
    on G1's columns, G2's mode-2 fibres and G3's rows."""
    tau, alpha = _rule()
    tt = inputs.tt_input(N_SMALL, ranks=(2, 3), seed=1)
    cols, tab = structured.tt_apply(tt, N_SMALL, H_SMALL, tau, alpha)
    dense = structured.tt_densify(cols, tab, len(tau), N_SMALL, 2, 3)
    phi, hf = apply.kron_apply_dense(structured.tt_to_full(tt, N_SMALL), H_SMALL, tau, alpha)
    assert apply.rel_l2(dense[0], phi) < 1e-13
    assert apply.rel_l2(dense[1:], hf) < 1e-13


def test_tt_equals_tucker2():
    """App. C: [[G2; G1, id, G3^T]] reproduces the TT entries a_ijk = G1(i) G2(j) G3(k)."""
    tt = inputs.tt_input((4, 5, 3), ranks=(2, 3), seed=2)
    full = structured.tt_to_full(tt, (4, 5, 3))
    q = 1
    ref = np.zeros((3, 5, 4))
    for i in range(4):
        for j in range(5):
            for k in range(3):
                ref[k, j, i] = tt.G1[q][i, :] @ tt.G2[q][:, j, :] @ tt.G3[q][:, k]
    assert np.allclose(full[q], ref, rtol=1e-14, atol=1e-14)


def test_structured_dft_lemmas():
    """Lemmas DFT_cp and DFT_tucker: the 3D DFT of a CP/Tucker tensor is the
    CP/Tucker tensor of the column-wise 1D DFTs of its factors."""
    cp = inputs.cp_input((6, 5, 4), rank=3, seed=7)
    full = structured.cp_to_full(cp, (6, 5, 4))[0]
    Fu = [np.fft.fft(cp.U[0][d], axis=0) for d in range(3)]
    via = np.einsum("r,xr,yr,zr->zyx", cp.lam[0], *Fu)
    assert np.allclose(np.fft.fftn(full), via, rtol=1e-12, atol=1e-12)
    tk = inputs.tucker_input((6, 5, 4), ranks=(2, 2, 3), seed=7)
    full = structured.tucker_to_full(tk, (6, 5, 4))[0]
    Fu = [np.fft.fft(tk.U[0][d], axis=0) for d in range(3)]
    via = np.einsum("abc,xa,yb,zc->zyx", tk.core[0], *Fu)
    assert np.allclose(np.fft.fftn(full), via, rtol=1e-12, atol=1e-12)


def test_circulant_embedding_is_toeplitz_product():
    """Sec. 4.2 with the padding length read as L = 2n: the circulant with first
    column [g_0..g_{n-1}, 0, g_{-(n-1)}..g_{-1}] restricted to n outputs is the
    Toeplitz product (convolution theorem, Sec. 4.1)."""
    rng = np.random.default_rng(0)
    n = 13
    g = rng.standard_normal(2 * n - 1)
    u = rng.standard_normal(n)
    c = np.concatenate([g[n - 1:], [0.0], g[:n - 1]])
    y = np.fft.irfft(np.fft.rfft(c) * np.fft.rfft(u, 2 * n), 2 * n)[:n]
    assert np.allclose(y, sinc.toeplitz(g) @ u, rtol=1e-13, atol=1e-13)


def test_term_table_columns():
    """Each CP term uses, per axis, the column of its own (q, k, l) with the
    derivative slot set only on the differentiated axis of h_d."""
    M, r = 3, 2
    tab = structured.term_table(M, r)
    assert tab.shape == (4, 3 * M * r, 3)
    for o in range(4):
        for q in range(3):
            for k in range(M):
                for l in range(r):
                    for d in range(3):
                        q_, rem = divmod(int(tab[o, (q * M + k) * r + l, d]), 2 * M * r)
                        s_, rem = divmod(rem, M * r)
                        k_, l_ = divmod(rem, r)
                        assert (q_, k_, l_) == (q, k, l)
                        assert s_ == (1 if o == d + 1 else 0)


# ---------------------------------------------------------------- bf16
def test_bf16_bits_match_torch_rne():
    """Round-to-nearest-even, checked against PyTorch's own float->bfloat16."""
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000).astype(np.float32),
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 3.0e-38,
                                  65504.0, 1e-10], dtype=np.float32)])
    ours = bf16.bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_bf16_known_ties():
    assert bf16.bf16_bits(np.float32(1.0)) == 0x3F80
    assert bf16.bf16_bits(np.float32(1 + 2 ** -8)) == 0x3F80        # tie -> even
    assert bf16.bf16_bits(np.float32(1 + 3 * 2 ** -8)) == 0x3F82    # tie -> even
    assert bf16.bf16_bits(np.float32(-2.0)) == 0xC000


def test_three_way_split_is_exact():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    hi, lo, lo2 = (bf16.bf16_value(p) for p in bf16.split(x, 3))
    assert np.array_equal((hi.astype(np.float64) + lo + lo2), x.astype(np.float64))
    hi2, lo_2 = (bf16.bf16_value(p) for p in bf16.split(x, 2))
    rel = np.abs((hi2.astype(np.float64) + lo_2) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -16


@pytest.mark.parametrize("parts,bound", [(2, 3e-5), (3, 1e-6)])
def test_split_products_accuracy(parts, bound):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((64, 128)).astype(np.float32)
    B = rng.standard_normal((128, 32)).astype(np.float32)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    got = bf16.split_matmul(A, B, parts).astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < bound


# cells of the n = 4096 uniform-cube pin: corners, face and edge centres,
# the centre, interior points
CUBE_CELLS_4096 = [(0, 0, 0), (4095, 4095, 4095), (0, 2048, 2048), (2048, 0, 4095), (2048, 2048, 2048),
                   (1234, 3000, 17), (4095, 2048, 1), (700, 701, 702)]


def uniform_cube_structured_values(F, m, cells):
    """phi, h_x, h_y, h_z at the given cells of the structured (CP) result for
    the uniform magnetization m: one rank-1 term per component whose columns
    are the output columns of constant inputs, i.e. the row sums of the
    Toeplitz factors (Eq. (kron_eval_cp) with all factor columns ones)."""
    n = (F.shape[2] + 1) // 2
    M = F.shape[1]
    out = np.zeros((len(cells), 4))
    for c, cell in enumerate(cells):
        for o in range(4):
            for q in range(3):
                for k in range(M):
                    v = m[q]
                    for d in range(3):
                        g = F[structured.type_of(q, d, structured.slot(o, d)), k]
                        v *= g[cell[d]:cell[d] + n].sum()   # sum over source cells j of g[i - j + n - 1]
                    out[c, o] += v
    return out


def test_uniform_cube_4096_structured_equals_exact_collocation():
    """n = 4096 per axis (unit cube), 64-node theorem-step rule (Thm.
    sinc_theo): the structured apply's values for a uniform magnetization
    equal the exact collocated potential and field of the uniformly
    magnetized cube (closed-form box kernels at the cell centres, the cell
    sum of the integral by additivity) to 1e-9 at corners, face and edge
    centres and interior cells.  This pins the operator at the structured
    path's full size to the exact collocation, not only to itself."""
    n = 4096
    h = 1.0 / n
    _t, tau, alpha = sinc.sinc_nodes(64, step_rule=1, h_min=h)
    F = sinc.scaled_factors(n, h, tau, alpha)
    m = np.array([0.3, -0.5, 0.8])
    got = uniform_cube_structured_values(F, m, CUBE_CELLS_4096)
    for c, cell in enumerate(CUBE_CELLS_4096):
        pt = (np.array(cell) + 0.5) * h
        K, N = exact.box_kernels_at_points(pt, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
        ref = np.concatenate([[K @ m], -N @ m])
        assert np.linalg.norm(got[c] - ref) <= 1e-9 * np.linalg.norm(ref), (cell, got[c], ref)
