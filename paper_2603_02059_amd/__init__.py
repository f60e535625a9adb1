"""TRAKNN hot path on MI355X: exact all-pairs kNN over length-L trajectories of
gridded fields (symmetric MFMA Gram, diagonal window recurrence, exclusion-zone
top-k rarity score, and its backward), behind the C ABI in ``include/traknn.h``.

Submodules are imported lazily: ``synth`` (seeded inputs, numpy only) never
loads the HIP library; ``traknn`` (the binding) does, and fails loudly if the
library has not been built.
"""
__all__ = ["synth", "traknn"]
