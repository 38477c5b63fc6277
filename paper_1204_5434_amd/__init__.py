"""MI355X-native propagator hot path of polymer field theory (arXiv:1204.5434).

The compute path is the HIP library ``libpft.so`` (C ABI in include/pft.h);
``binding`` marshals torch tensors into it.  ``inputs`` draws the seeded
synthetic workloads.
"""
__all__ = ["binding", "inputs"]
