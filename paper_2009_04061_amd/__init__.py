"""GPA hot path on MI355X: sample aggregation, reaching definitions, the
instruction blamer and the scope-level speedup estimators behind a C-ABI
library of hand-written HIP kernels for gfx950.

Importing the package loads nothing; ``paper_2009_04061_amd.gpa`` is the
binding to the compiled library and ``paper_2009_04061_amd.synth`` the
seeded input generator.
"""
