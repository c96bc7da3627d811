"""Seeded synthetic inputs shared by the decoder tests, the benchmark and the oracle checks.

Codes (parity-check matrices), systematic GF(2) encoding of random information
bits, and BPSK/AWGN channel LLRs.  The module holds no decoding arithmetic.
"""
from . import channel, codes, gf2, workloads  # noqa: F401
