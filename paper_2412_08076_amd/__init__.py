"""MI355X (gfx950) implementation of the long-step Richardson(m) / NAG-Richardson(m)
hot path of arXiv 2412.08076.

The compute lives in librm.so (HIP kernels behind the C ABI of include/rm.h).
``paper_2412_08076_amd.rm`` marshals torch tensors into those calls and
``paper_2412_08076_amd.autograd`` wraps them for training.  Importing this
package does not load the library; the first call does, and fails loudly when
it has not been built.
"""
