"""MI355X-native VDI generation and compositing (arXiv 2206.14503).

The hot path is libvdi.so (HIP kernels for gfx950 behind the C ABI declared in
include/vdi.h); `paper_2206_14503_amd.vdi` is its Python binding and
`paper_2206_14503_amd.synth` holds the seeded synthetic inputs.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["vdi", "synth"]
