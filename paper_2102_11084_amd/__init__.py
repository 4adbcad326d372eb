"""MI355X-native voxel-grid point-cloud downsampling (arXiv 2102.11084).

The compute path is the HIP library `libvg.so` (kernels for gfx950 behind a C
ABI); `paper_2102_11084_amd.vg` is the thin Python binding over it.  Importing
the package loads nothing; the binding loads the library on first use and
raises if it is missing.
"""
