"""Build the HIP library in-tree if it is missing (CPU test runs only)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_1808_08645_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
