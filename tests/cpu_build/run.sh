#!/bin/bash
# Threaded CPU build of the library (host code and kernel sources compiled for
# the host under AddressSanitizer and UBSan; one OS thread per GPU thread where
# a kernel synchronises) and the checks in check.py.  CPU only, no GPU; about
# 7 minutes to compile.  Usage: bash tests/cpu_build/run.sh [BUILD_DIR [CHECK...]]
set -euo pipefail
HERE=$(cd "$(dirname "$0")" && pwd)
OUT=${1:-$HERE/../../_build/cpu_build}
shift || true
mkdir -p "$OUT"
python3 "$HERE/extract.py" "$OUT"
CXX=${CXX:-/opt/rocm/llvm/bin/clang++}
"$CXX" -std=c++20 -O1 -g -fPIC -shared -fsanitize=address,undefined -fno-omit-frame-pointer \
    -I "$OUT" -I "$HERE" -include "$HERE/hip/hip_runtime.h" \
    "$HERE/harness.cpp" "$OUT/pf_api.cpp" -o "$OUT/libcpu.so" -lpthread
ASAN_RT=$("$CXX" -print-file-name=libclang_rt.asan-x86_64.so)
ASAN_OPTIONS=detect_leaks=0 LD_PRELOAD="$ASAN_RT" python3 "$HERE/check.py" "$OUT/libcpu.so" "$@"
