"""paper_2207_01834_amd -- ParGeo's kd-tree hot path on AMD Instinct MI355X.

GPU kd-tree construction and batched k-nearest-neighbour search (static and
BDL-tree forms) behind the C ABI of ``libpargeo_hip.so`` (see
``include/pargeo_hip.h``).  The Python layer only marshals arguments.

Submodules are imported lazily so that ``datagen`` (seeded inputs) can be
used without loading the GPU library.
"""

__all__ = ["kdtree_build", "KdTree", "BDLTree", "B1Tree", "B2Tree", "lib"]


def __getattr__(name):
    if name in ("kdtree_build", "KdTree", "BDLTree", "B1Tree", "B2Tree", "lib", "PargeoError", "RangeError"):
        from . import _binding
        return getattr(_binding, name)
    raise AttributeError(name)
