"""The GPU kernels' smoothing tables are generated, not hand-edited.

csrc/gen_smoothing.py derives the Taylor coefficients of F1..F4 and G2, G4 in
exact rational arithmetic, the far-field cutoffs, and the erfcx fits used by
the near-field branch (checking each fit's error in its target precision);
the committed smoothing_coeffs.h must be exactly its output.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_10749_amd", "csrc")


def test_smoothing_header_is_the_generator_output():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_smoothing.py")], capture_output=True, text=True,
                         check=True, timeout=300).stdout
    with open(os.path.join(CSRC, "smoothing_coeffs.h")) as f:
        assert f.read() == out
