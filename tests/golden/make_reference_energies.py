"""Recompute the numeric entries of reference_energies.txt (calls only oracle/exact.py)."""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import lrh_workloads as W  # noqa: E402
from oracle import exact  # noqa: E402

if __name__ == "__main__":
    print("tfim_chain_n16_E0", repr(exact.tfim_open_chain_E0(16, 1.0, 0.5)))
    print("heisenberg_chain3_E0", repr(exact.ground_energy(W.heisenberg_chain(3))))
    print("tfim_torus4x4_h2.5_E0", repr(exact.ground_energy(W.tfim_growing_clusters(4, 2.5, 0))))
