"""paper_2405_17696_amd -- batched 2D Helmholtz solves on gfx950 (MI355X).

Flexible GMRES preconditioned by a shifted-Laplacian V-cycle or by an
encoder-solver U-Net, network training, and the adjoint misfit gradient, all
in hand-written HIP kernels behind the C ABI of include/helm.h.  Importing the
package loads nothing; the first call into `api` loads libhelm.so and raises
if it is missing.
"""
__all__ = ["api", "synth"]
