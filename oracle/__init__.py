"""Reference (oracle) implementation of higher-order motif counting.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, CPU implementation
of what the product computes, written from the paper's definitions and
algorithms.  Only the test-suite, the smoke check and the benchmark's CPU
baseline leg may import it.  It shares no code with the HIP library: the two
meet only through the seeded input generators in ``workloads``.

Modules
-------
classes   isomorphism classes of k-node patterns (Section 4.3, Fig. 3a)
brute     brute force over all k-subsets: the plain definition (Section 3)
core      literal Algorithms 2, 3 and 4 in C, through ctypes
philox    Philox4x64-10 counter-based generator (Salmon et al., SC'11)
stats     null-model invariants, z-scores, error measures
mlp       reference forward/backward of the learned proposal's MLP
"""
