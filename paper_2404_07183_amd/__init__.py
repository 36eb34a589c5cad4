"""MI355X (gfx950) library for pairwise integrated combinations of piecewise
constant functions: L_p distance and L2 Gram matrices, batched and
differentiable (arxiv 2404.07183, Sections 2-3).

The compute path is the C-ABI HIP library ``libpcf.so`` (``include/pcf.h``);
``paper_2404_07183_amd.api`` wraps it for PyTorch tensors. Importing this
package does not load the library; the first call does, and fails loudly if
it is not built.
"""
