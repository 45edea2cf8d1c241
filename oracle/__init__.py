"""CPU oracle for the encrypted GCN layer X' = A X W under RNS-CKKS.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code,
tables or constants with the GPU library: it derives its own primes, roots and
base-conversion constants from their definitions, with Python integers or the
plain C of ``core.c`` (128-bit products, no lazy reduction).

Modules:
  ntheory   primes, roots of unity, CRT (Python integers)
  params    CKKS parameter set (paper Sec. 2.1)
  sampler   ChaCha20 streams -> uniform / ternary / CBD(21) polynomials
  ckks      keygen, encrypt, decrypt, rescale, key switching, rotation,
            plaintext and scalar multiply-accumulate, ct x ct multiply
  encoding  canonical-embedding encode / decode
  gcn       the FP64 GCN the encrypted layer must reproduce (Sec. 2.2)
  planner   packing cost model, aggregation-mode rule, node-order
            optimisation (Alg. 1), shift routing
  simulate  slot-level simulator of a plan on cleartext vectors
  execute   the plan executed on oracle ciphertexts
"""
