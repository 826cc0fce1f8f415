"""Plain, slow, FP64 CPU oracle for adaptive block compressive sensing.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never calls it and shares no code, table
or constant with it.

Modules:
  abcs     - geometry, budget scalars, 2D-DCT, zigzag order, BBV and DD
             statistics, capped apportionment, sensing, masked inverse DCT
             (Sections IV-V, Algorithms 1-2, eqs 16-23, 26).
  ida      - the IDA post-processing loop (Section VI, eqs 13, 15, 25, 28).
  metrics  - PSNR and SSIM.
  bm3d     - the plain BM3D denoiser used inside IDA.
  cnn      - the learned convolutional denoiser (forward, backward, Adam).

Parity status of each function is stated in its module header.
"""
