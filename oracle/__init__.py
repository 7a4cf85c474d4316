"""The oracle: a plain, byte-oriented CPU AES (FIPS-197; ECB and CTR).

Test infrastructure only.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import it; the GPU package never does.
"""
