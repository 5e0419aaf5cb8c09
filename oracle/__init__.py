"""CPU FP64 oracle of the power-Doppler reconstruction path.

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the CPU-baseline leg of
the benchmark may import this package.  It is independent of the HIP path:
it never imports or loads the GPU library, and the GPU library never calls it.
The two share only the seeded input generators in `fqscene`.

Modules
  native   ctypes front-end of fq_oracle.c (RF synthesis, rf2iq, DAS; plain C, FP64)
  clutter  Casorati Gram, Hermitian eigendecomposition, rank selection (knee),
           SVD clutter filter and power Doppler (numpy, FP64)
  bf16     bit-exact round-to-nearest-even BF16 and the split-BF16 Gram emulation
  lcf      learned slow-time convolutional clutter filter: forward, backward, Adam
  pipeline end-to-end chain scene -> RF -> IQ -> PD for small workloads
"""
