"""MI355X (gfx950) implementation of the halftoning method of "Efficient
Halftoning via Deep Reinforcement Learning" (Jiang et al., arXiv 2304.12152).

The compute lives in libhalftone.so (hand-written HIP, C ABI in
include/halftone.h); `binding` exposes its entry points under the same names,
`autograd` wraps them as torch.autograd Functions, `synth` makes seeded
synthetic inputs. Importing the package loads nothing.
"""
__version__ = "1.0.0"
