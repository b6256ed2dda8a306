"""Plain, slow FP64 CPU oracle of the groupwise Tucker compression and compressed-domain SINR.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its Python
binding) imports, links or calls this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code, tables or helpers with the GPU path;
only the seeded input generator (package `synthgen`) is common to both sides.

Modules
  tensor   -- inner product, norm, mode-n unfolding and mode-n product (Section 2.3)
  tucker   -- HOSVD initialisation, the alternating factor updates of the groupwise model,
              the optimal core, the objective, reconstruction (Sections 2.3, 3.2)
  sinr     -- SVD precoder, MMSE receive filter, covariance, signal power and SINR on full
              and compressed channels, and the compressed-domain Woodbury forms (Sections 2.2, 3.3)
  metrics  -- NMSE, SINR error in dB, mean relative SINR error, storage ratios (Section 4)
  grad     -- FP64 gradients of the compressed SINR and of reconstruction (torch autograd on CPU)

Every function is pinned by a test under tests/ that checks it against something other than
itself (closed forms, special cases that reduce to a library routine, invariants, brute force,
the storage column of the paper's Table 1).  Parity unpinned: none of the functions here;
the paper's own R_t and e_c columns of Table 1 are not reproducible without its 3GPP data.
"""
