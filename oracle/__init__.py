"""AIRPF CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, sequential implementations of what the AIRPF hot path computes,
used to check the HIP library.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.  See oracle/orc_airpf.c for the algorithm and its citations.
"""
