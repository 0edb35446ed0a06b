"""FP64 CPU oracle of the PDCS LP method -- test infrastructure only.

Used by tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py.
The product path (paper_2603_15504_amd) never imports it.
"""
