"""FP64 CPU oracle for the sliCQ transform (Holighaus, Doerfler, Velasco, Grill,
"A framework for invertible, real-time constant-Q transforms").

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
GPU library is checked against. Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it. The product library
(``paper_1210_0084_amd``) never imports, links or runs anything in here, and
this package imports nothing from the product library: the two share only the
seeded input generators in ``workloads``.

Layout
------
``plan``       constant-Q band design (Section 3, Table 1), lattice and
               painless dual (Proposition 2), Tukey slicing windows and their
               dual (Section 4.3, equations BUPU and dualwincond).
``transform``  sliCQ analysis and synthesis (Algorithms 1-4) with NumPy FFTs
               as steps, the adjoint of analysis, the linear (streaming) form.
``brute``      the plain definitions: atoms T_{n a_k} F^{-1} g_k, coefficients
               as inner products (equation CQ_coeff), the dense frame operator
               (equation frameop) and dual atoms (equation candual).
``layers``     the 2-layer array of Algorithm 3, the sliCQ spectrogram, dB
               masks and band transposition (Sections 4.3 and 6).
``fullnsgt``   the full-length CQ-NSGT on the same band windows, the SNR of
               Section 5.3 and the bound of Proposition 4.

Every function that has no independent pin says "parity unpinned" in its
docstring; all functions here are pinned by tests under ``tests/`` marked
``not gpu``.
"""
from .plan import OraclePlan, BandTable, plan_from_tables, q_factor  # noqa: F401
from .transform import (analyze, synthesize, adjoint, analyze_full, synthesize_full,  # noqa: F401
                        num_slices, padded_length, analyze_stream, synthesize_stream, pack, unpack,
                        analyze_slices, synthesize_slices, synthesize_adjoint, pack_full, unpack_full)
from . import layers, fullnsgt  # noqa: F401
from . import brute  # noqa: F401
