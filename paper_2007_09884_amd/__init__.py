"""MI355X-native OPMM estimation (arXiv 2007.09884).

The hot path -- simulate the oculomotor plant for very many candidate OPC
vectors, score each against a recorded saccade, argmin, refine -- runs in
hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/opmm.h``.  ``paper_2007_09884_amd.opmm`` is the thin Python binding.
Importing the package does not load the library; ``synth`` is importable
without a GPU.
"""
