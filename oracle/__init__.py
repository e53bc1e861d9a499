"""Plain, slow, obviously correct CPU oracle for the Pauli-rotation hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call, link or execute anything
under ``oracle/``.  The library (``paper_2504_17881_amd``) never does, and the
oracle never imports the library: the two share no code.  Their only common
source is the seeded input generator package ``synth``, which holds none of
the method's arithmetic.

Contents:
  * ``statevector``: rotation sequences applied in the scatter form, FP64, in
    numpy and in plain C (``oracle.c``, built by ``oracle/build.py``);
    compensated overlap and norm.
  * ``schedules``: the product-formula schedules (first- and second-order
    Trotter, qDRIFT, the partially randomised formula), re-expanded from the
    paper's definitions, with the SplitMix64 generator written from its
    published definition.
  * ``pauli``: the letter <-> two-mask encoding of Pauli strings.

Every function names the passage of the paper it follows.  Pins that tie the
oracle to something other than itself live in ``tests/test_oracle_pins.py``.
Parity status: every function here is pinned (see that file); none is
"parity unpinned".
"""
