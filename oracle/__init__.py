"""TEST INFRASTRUCTURE ONLY: the CPU oracle for the pair-distance histogram.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library never imports it.
See ``dh_oracle.c`` for the definition it implements and its citations.
"""
from .oracle import (  # noqa: F401
    BOX_NONE, BOX_ORTHO, BOX_TRICLINIC, IMAGES_PAPER, IMAGES_27, IMAGES_125,
    OracleResult, build, histogram, frame_histogram, pair_t, min_width, max_threads, load,
    edge_window,
)
