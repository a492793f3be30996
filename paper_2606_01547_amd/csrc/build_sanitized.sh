#!/bin/sh
# Host-sanitized builds of libjt and of the server stress driver
# (tests/native/server_stress.cpp), for CPU runs against the simulated server:
#   build_sanitized.sh asan OUTDIR   AddressSanitizer + UndefinedBehaviorSanitizer
#   build_sanitized.sh tsan OUTDIR   ThreadSanitizer
# Only host code is instrumented (each -fsanitize= sits behind -Xarch_host);
# the gfx950 device code is compiled as in build.sh.  Writes
# OUTDIR/libjt_<kind>.so and OUTDIR/server_stress_<kind>.
set -e
KIND=$1
OUT=$2
[ -n "$KIND" ] && [ -n "$OUT" ] || { echo "usage: $0 asan|tsan OUTDIR" >&2; exit 2; }
HERE=$(cd "$(dirname "$0")" && pwd)
ROOT=$(cd "$HERE/../.." && pwd)
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
CLANGXX=${CLANGXX:-/opt/rocm/llvm/bin/clang++}
case "$KIND" in
  asan) SAN="-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=undefined"
        LINK="address,undefined" ;;
  tsan) SAN="-Xarch_host -fsanitize=thread"
        LINK="thread" ;;
  *) echo "unknown kind $KIND" >&2; exit 2 ;;
esac
mkdir -p "$OUT"
FLAGS="--offload-arch=gfx950 -O1 -g -fno-omit-frame-pointer -std=c++17 -fPIC -shared -Wno-unused-command-line-argument -Xclang -target-feature -Xclang -packed-fp32-ops"
$HIPCC $FLAGS $SAN -o "$OUT/libjt_$KIND.so" "$HERE"/*.hip "$HERE"/*.cpp
# the driver carries the sanitizer runtime; the library resolves against it
$CLANGXX -O1 -g -fno-omit-frame-pointer -std=c++17 -fsanitize=$LINK -D__HIP_PLATFORM_AMD__ -I"$ROOT/include" \
  -I/opt/rocm/include -o "$OUT/server_stress_$KIND" "$ROOT/tests/native/server_stress.cpp" \
  -L"$OUT" -ljt_$KIND -Wl,-rpath,"$OUT" -lpthread
