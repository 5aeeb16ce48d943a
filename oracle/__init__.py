"""FP64 CPU oracle of the distributed deblurring method (Mourya et al.,
"Distributed Deblurring of Large Images of Wide Field-Of-View").

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, obviously-correct
NumPy implementation that the tests, the smoke check and the benchmark's CPU
baseline compare the HIP library against.  The product path never imports,
calls or falls back to anything in this package, and this package shares no
code with the HIP library (only the seeded input generators are common).

Modules:
  layout   -- tiles, supports, consensus weights omega, PSF-interpolation tents
              (Sections II-B and III-A, Fig. 1)
  operator -- the per-tile shift-variant blur H_t and its adjoint by direct
              spatial convolution (Section II-B), the global operator used to
              simulate data (Eq. (2)), and an FP64 FFT backend
  prior    -- smoothed total variation and Huber regularisers (Section IV-A)
  solver   -- Local-Solver (projected gradient on the prox subproblem, or its
              FISTA-accelerated form),
              consensus by the Lemma of Section III-B, the D-R outer loop of
              Algorithm 1, residual and output assembly
  minimiser-- the result oracle: a direct minimiser of the consensus problem
              Eq. (4) for tiny images, and dense closed-form solves
  cnn      -- the warm-start network (forward / backward, BF16 rounding, Adam)
  warm     -- the warm start around the network: tile scale and input,
              network start, and the per-tile gradient-map fallback judge

Parity unpinned: nothing in the deblurring path.  The paper's SNR/SSIM figures
need its natural test images and are not reproduced.
"""
