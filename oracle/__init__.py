"""FP64 CPU oracle for the discrete-cosine tensor Krylov methods.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
numpy implementation of what the HIP library computes.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP library (no kernels,
no helpers, no tables): it builds its own transform matrices from the paper's
closed forms and follows the paper's algorithms step by step.

Layout convention: a third-order tensor A in R^{n1 x n2 x n3} is stored as a
numpy array of shape (n3, n1, n2), i.e. frontal slice k is ``A[k]``.

Modules
  tube      -- the DCT matrix C_n (eq. dft1), th(v) (eq. dft5), mat/ten
               (Sec. 2.2), the mode-3 transform matrix M (Remark 2.1)
  cprod     -- the c-product (Definition of Sec. 2.2, Algorithm 1), its exact
               adjoint, and the one/two-sided operators of eq. (2)
  krylov    -- global Golub-Kahan (Algorithm 4), DC-LSQR (Algorithm 6),
               global Arnoldi (Algorithm 2), DC-GMRES(m) (Algorithm 3)
  tikhonov  -- projected Tikhonov by SVD and GCV (eqs. leastsq, normeq2, gcv2)
  metrics   -- relative error and SNR (Sec. 4)
  mlp       -- the learned stopping index / regularisation parameter: features
               from the first GKB steps, the 16-64-64-2 GELU network with
               bfloat16-rounded weights, its gradients, loss and Adam step
"""
