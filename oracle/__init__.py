"""CPU oracle for the hierarchical matrix-vector product.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the CPU
baseline leg of bench.py may import, call, link or execute anything under
oracle/.  The product path (the HIP library and its Python binding) never
does, and must fail loudly when its extension is missing.

A plain, slow, float64 implementation written from the paper's definitions
(Kriemann, "Floating Point Compression of Hierarchical Matrix Formats and its
Impact on Matrix-Vector Multiplication"): cluster and block trees
(Def. 2.1, 2.2), the exact-cover validator, the dense kernel product (Sec.
2.1), the H / uniform-H / H^2 products (Sec. 3, Alg. 1, 3-7, eq. 4-5) and
the storage formats (Table 1, Sec. 4).  It shares no code with the GPU path;
both consume the same seeded inputs from the `synth` package.
"""
