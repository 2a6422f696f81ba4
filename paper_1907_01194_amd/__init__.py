"""MI355X-native hot path of the manifold-optimisation ground-state solver for
spin-F Bose-Einstein condensates (energy, Riemannian gradient, Hessian-vector
products, retractions and the regularized Newton driver) as a HIP library with
a C ABI (``include/gpe.h``) and a thin ctypes binding (``binding``).

The binding is imported lazily: ``import paper_1907_01194_amd`` does not load
the shared library; the first use of ``binding`` does, and fails loudly if the
library has not been built.
"""

__all__ = ["binding", "workloads", "autograd"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
