"""MI355X library for the encrypted GCN layer X' = A_hat X W under RNS-CKKS
(FicGCN, arXiv 2506.10399).

  ficgcn   ctypes binding of the C ABI (include/ficgcn.h), one method per entry point
  graph    client/server-side data preparation: normalised adjacency in CSR,
           the client's slot layouts, reading outputs
  build    hipcc build of libficgcn.so for gfx950
"""
