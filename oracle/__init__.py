"""Plain FP64 CPU oracle for the eHDG iteration.

TEST INFRASTRUCTURE ONLY: used by tests/, by __graft_entry__.smoke() and by the
cpu_baseline leg of bench.py.  The product path never imports it and shares no
code, headers, tables or helpers with it.
"""
