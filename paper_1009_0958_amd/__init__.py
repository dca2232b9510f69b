"""Order-statistics directional filters (BVDF, DDF) on AMD Instinct MI355X.

The compute path is the HIP library ``libodf.so`` (C ABI in include/odf.h);
``paper_1009_0958_amd.odf`` is its Python binding and
``paper_1009_0958_amd.synth`` the seeded synthetic-input generator.
"""
