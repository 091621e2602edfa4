"""CPU reference ("oracle") for the stray-field operator of Exl et al.,
"FFT-based Kronecker product approximation to micromagnetic long-range
interactions" (arXiv 1212.3509).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library, its Python binding or
its benchmark's timed path imports this package; only the test-suite, the
smoke check and the benchmark's CPU-baseline leg do.  It is plain, slow,
float64 NumPy/SciPy code written so that each function can be checked against
the paper by eye.  It shares no code with the HIP implementation: the only
common module is the seeded input generator ``paper_1212_3509_amd.inputs``,
which holds no arithmetic of the method.

Modules
  exact       closed-form cell kernels (potential and demagnetizing tensor),
              the tau-integral form of Eq. (conv_op) by adaptive quadrature,
              and brute-force face cubature (independent third route)
  sinc        quadrature nodes and the 1D factors of Cor. kron_op / Eq. (conv_pot)
  apply       collocated potential/field (Eq. (coll)) by FFT convolution or direct
              sums, and the Kronecker-form apply with dense Toeplitz factors
  structured  the Kronecker operator applied to CP, Tucker and TT inputs
              (Eqs. (kron_eval_cp), (kron_eval_tuck); App. C) with dense factors
  bf16        round-to-nearest-even bfloat16 splitting by integer bit operations
  mlp         float64 multilayer perceptron with hand-written backward and Adam
  smooth      exact potential of a smooth magnetization by singularity
              subtraction (reference for Lemma conv_coll / Fig. fig_err)
  quadrule    shortened rules, their operator-norm certificate and fit
  recompress  HOOI recompression of CP tensors (Alg. HOOI)
  fftconv     the Kronecker operator as one 3D FFT convolution
  nonuniform  dense 1D factors of non-uniform tensor grids
  tucker      Alg. scpot_fft_tucker (kernel compression, Fourier-space
              Tucker Hadamard products, approximate summation), TT rounding

Readings of the paper that the oracle adopts are listed in each module header.
"""
