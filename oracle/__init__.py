"""FP64 CPU oracle for the compressed-DMD hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the CPU
baseline leg of bench.py.  The product library and its Python binding never import,
call or link anything here, and this package imports nothing from the product.
"""
