"""krt: polarized Kerr ray tracing on AMD MI355X (gfx950).

The compute path lives in the C-ABI library ``libkrt.so`` built from
``csrc/``; ``paper_2302_02733_amd.krt`` is its thin ctypes binding and
``paper_2302_02733_amd.workloads`` holds the seeded synthetic inputs.
Submodules are imported explicitly so that loading the input generators does
not load the GPU library.
"""
