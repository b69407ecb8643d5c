"""CPU reference for the screened PT2 energy -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it, and it shares no code
with the GPU library.

* `oracle.ref`   -- ctypes front end of the brute-force C++ reference
                     (`pt2_oracle.cpp`);
* `oracle.dense` -- a tiny full-CI checker that builds H by explicit
                     second-quantised operator application, used to pin the
                     C++ reference on small systems.
"""
