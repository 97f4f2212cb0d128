"""CPU oracle for the Combined Sieve -- test infrastructure, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
or execute anything in this package.  The HIP library never calls it and it never calls the HIP
library: the two share no code, headers or tables.

Contents
  plain.py            pure-Python literal definition (bignum N mod p per interval), tiny cases
  csieve_oracle.c     the same plain per-interval sieve in C with OpenMP over rows, for sizes
                      the Python version cannot reach
  coracle.py          ctypes wrapper of the C oracle
  build.py            compiles csieve_oracle.c with gcc

Every function states the passage of the paper it follows.  Pins (tests/test_oracle_pins.py)
tie it to numbers printed in the paper, closed forms and brute force.  Parity status of each
function: pinned (see the pin tests); nothing here is "parity unpinned" except the statement
that C3 rows beyond the sampled ones are unchecked, which concerns the HIP path, not the oracle.
"""
