"""MI355X (gfx950) HMM forward log-likelihood library for long tremor chains.

The compute path lives in the HIP shared library built from ``csrc/`` and is
reached through the C ABI declared in ``include/hmm.h``; ``binding`` marshals
torch tensors into that ABI.  ``synth`` draws seeded synthetic workloads.
Submodules are imported lazily so that ``synth`` can be used without the
compiled library.
"""
__all__ = ["binding", "synth"]
