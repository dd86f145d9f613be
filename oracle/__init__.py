"""FP64 direct-summation oracle for the FCBM-EC peridynamic operators.

Test infrastructure only: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py, never by the product package.
"""
