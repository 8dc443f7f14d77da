"""MI355X-native preconditioned iPEPS step (arXiv:2511.09546).

The compute path is the C-ABI library libipeps.so (hand-written gfx950
HIP kernels); ``binding`` marshals arguments to it.  Importing the package
does not load the library; ``binding.load()`` does, and raises if it has not
been built.
"""
__all__ = ["binding", "inputs", "build"]
