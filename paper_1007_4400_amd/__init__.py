"""MI355X-native seeded solver for sequences of dense complex Hermitian
generalized eigenproblems A x = lambda B x (lowest nev pairs).

``paper_1007_4400_amd.gevp`` is the ctypes binding of the HIP library
``libgevp.so``; ``paper_1007_4400_amd.synth`` builds seeded input sequences.
"""
__all__ = ["gevp", "synth"]
