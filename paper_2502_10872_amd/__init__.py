"""MI355X-native corotational hinge plate/shell bending hot path.

The compute path is the HIP library built from csrc/ (C ABI declared in
include/shell.h); `paper_2502_10872_amd.shell` is its thin ctypes binding and
`paper_2502_10872_amd.inputs` the seeded synthetic workload generators.
"""
