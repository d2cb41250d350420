"""Loader for the error tables under tests/golden (values printed in the paper)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            b, g, M, N, e = line.split()
            rows.append((float(b), float(g), int(M), int(N), float(e)))
    return rows
