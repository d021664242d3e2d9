"""Polya-urn LDA (doubly sparse partially collapsed Gibbs sampler) on MI355X.

Submodules are imported on demand: ``synth`` (seeded synthetic corpora) has no
dependency on the compiled library; ``pulda`` is the binding to libpulda.so.
"""
__all__ = ["synth", "pulda", "server"]
