"""FP64 / exact-integer CPU oracle for Neural Texture Block Compression (BC1 and BC4).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the package smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never calls it, and it shares
no code, tables or helpers with the GPU library.

Modules:
  bc       BC1/BC4 block format: palettes, decode, pack/unpack, the integer reference encoders.
  grid     Multi-resolution 2-D feature grids: block-centre sampling, bilinear blend, per-level QAT.
  lowp     Rounding to bfloat16 and to FP8 E4M3 (OCP), used to emulate the reduced-precision paths.
  mlp      The MLP trunk and its backward pass.
  ntbc     Heads -> endpoint quantisation -> index selection -> packing; the training losses with the
           straight-through estimator; Adam and the learning-rate schedule; one training step.
  metrics  PSNR, block identity, decision margins for the tie classification.

Floating-point work is done in float64 unless a function says otherwise.  Integer decisions (BC codes,
indices, quantised values) use Python/NumPy integers, or are taken in float32 where the function is the
checker for a float32 decision of the GPU path (the argument ``precision="f32"``).
"""
