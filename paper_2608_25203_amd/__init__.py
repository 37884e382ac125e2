"""MI355X-native Zakharov/HOS wave step: HIP kernels behind a C ABI.

The compute path is the shared library built from ``csrc/`` (``libzk.so``);
``paper_2608_25203_amd.zk`` is a thin ctypes binding with the same entry-point
names.  ``inputs`` holds the seeded synthetic input generators.
"""
