#!/bin/sh
# Builds the CPU reference library (test infrastructure only).  The library is
# written to a temporary name and renamed, so a process that has the old one
# loaded keeps a valid mapping.
set -e
cd "$(dirname "$0")"
g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared \
    pt2_oracle.cpp alias_oracle.cpp -o liboracle_pt2.so.tmp -lquadmath
mv liboracle_pt2.so.tmp liboracle_pt2.so
