"""Test infrastructure: the FP64 CPU oracle (see oracle.py). Not part of the product path."""
