"""CSS linear-scaling density matrix on MI355X (gfx950).

The compute path is the C-ABI library `libcss.so` built from `csrc/`; the
Python binding in `css.py` only marshals torch device tensors into it.
`synth` makes the seeded synthetic water-like workloads.
"""
