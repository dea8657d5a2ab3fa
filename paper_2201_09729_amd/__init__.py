"""MI355X (gfx950) implementation of the hot path of distillation low-mode
averaging (arXiv:2201.09729): batched Wilson-clover solves, the spatial
Laplacian eigensolver, the distillation projector and the correlator
contractions, behind the C ABI of include/dlma.h.  ``dlma`` is the Python
binding; ``synth`` draws the synthetic inputs."""
