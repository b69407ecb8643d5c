#!/bin/sh
# Builds the CPU reference library (test infrastructure only).
set -e
cd "$(dirname "$0")"
g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared \
    pt2_oracle.cpp -o liboracle_pt2.so -lquadmath
