"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds none of BlockBP's arithmetic (no contraction, no message
passing): only random site tensors, closed-form special states and a simple
update imaginary-time generator that produces physical-looking site tensors.
"""
