#!/bin/sh
# Builds libshci_pt2.so for gfx950 in this directory.
set -e
cd "$(dirname "$0")"
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
$HIPCC --offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared \
  -ffp-contract=off -fno-fast-math \
  -Xclang -target-feature -Xclang -packed-fp32-ops \
  -Wall -Wno-unused-function -Wno-unused-variable \
  csrc/api.hip csrc/tables.hip -o libshci_pt2.so.tmp
mv libshci_pt2.so.tmp libshci_pt2.so
