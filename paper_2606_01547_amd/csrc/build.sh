#!/bin/sh
# Builds libjt.so for gfx950 in-tree.  Usage: build.sh [output]
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
OUT=${1:-$HERE/../libjt.so}
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
FLAGS="--offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared -Wall -Wno-unused-command-line-argument -Xclang -target-feature -Xclang -packed-fp32-ops"
$HIPCC $FLAGS -o "$OUT.tmp" "$HERE/kernels.hip" "$HERE/adjoint.hip" "$HERE/fft.hip" "$HERE/linear.hip" "$HERE/noalloc.hip" "$HERE/calib.hip" "$HERE/jt_api.cpp" "$HERE/jt_params.cpp" \
  "$HERE/jt_ops.cpp" "$HERE/jt_grad.cpp" "$HERE/jt_server.cpp" "$HERE/jt_fit.cpp"
mv "$OUT.tmp" "$OUT"
