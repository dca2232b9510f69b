"""Order-statistics directional filters (BVDF, DDF) on AMD Instinct MI355X.

Placeholder: the GPU binding is added with the C-ABI library.
"""
