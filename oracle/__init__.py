"""CPU oracle for the PDX K-nearest-neighbour scan -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct FP64 implementations of what the GPU path
computes, written from the paper (Kuffo, Krippner, Boncz: "PDX: A Data
Layout for Vector Similarity Search", SIGMOD 2025) and checked against
closed forms, invariants, brute force and library routines in
``tests/test_oracle_*.py``.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import or run anything in this package.  The product
library (``paper_2503_04422_amd``) never imports it, and this package
never imports the product: the two share no code.  Inputs come from the
seeded generators in ``synth`` (random numbers only).

Modules
-------
exact     Exact KNN by definition (Section 2.1), numpy and a plain C build.
pdxearch  Step-by-step PDXearch (Section 4) with the PDX-BOND order and
          bound (Section 5) and with the ADSampling test (Section 2.3),
          plus the IVF-flat reference (Section 2.1).
rotation  Random orthogonal rotation (ADSampling, Section 2.3).
kmeans    Lloyd k-means (IVF, Section 2.1) and index invariants.
layout    The PDX layout by definition (Section 3, the kernel listing).
lowp      BF16 / FP8-e4m3 storage codes and their decode.
mlp       FP64 forward/backward of the learned pruning network.
"""
