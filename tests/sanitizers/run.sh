#!/bin/bash
# CPU-only sanitizer runs (no GPU needed):
#  1. the oracle built with AddressSanitizer + UBSan (g++), its pin tests;
#  2. libmcspect with the sanitizers on its host code only (hipcc
#     -Xarch_host; device code unchanged), the C-ABI host tests.
# Builds go to $OUT (default /tmp/mcspect_san); exits with the first failure.
set -eu
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
OUT=${OUT:-/tmp/mcspect_san}
mkdir -p "$OUT/host" "$OUT/pkg/paper_2105_13324_amd"

g++ -O1 -g -fno-omit-frame-pointer -fsanitize=address,undefined -fno-sanitize-recover=undefined \
    -std=c++17 -shared -fPIC -pthread "$ROOT/oracle/mc_oracle.cpp" -o "$OUT/liboracle_san.so"
LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)" \
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 \
    python3 "$ROOT/tests/sanitizers/oracle_pins.py" "$OUT/liboracle_san.so"

SRC="$ROOT/paper_2105_13324_amd/csrc"
for f in api staging transport adjoint sysmat cfd cgsm compose; do
    /opt/rocm/bin/hipcc -O1 -g -std=c++17 -fPIC --offload-arch=gfx950 \
        -Xclang -target-feature -Xclang -packed-fp32-ops \
        -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer \
        -w -I "$ROOT/include" -I "$SRC" -c "$SRC/$f.hip" -o "$OUT/host/$f.o"
done
/opt/rocm/bin/hipcc -shared -fPIC --offload-arch=gfx950 -Xarch_host -fsanitize=address \
    -Xarch_host -fsanitize=undefined -shared-libsan "$OUT"/host/*.o -o "$OUT/pkg/paper_2105_13324_amd/libmcspect.so"
cp "$ROOT/paper_2105_13324_amd/__init__.py" "$OUT/pkg/paper_2105_13324_amd/"
RT=$(ls /opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)
LD_PRELOAD="$RT" ASAN_OPTIONS=detect_leaks=0:abort_on_error=1:halt_on_error=1 \
UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 \
    python3 "$ROOT/tests/sanitizers/abi_host.py" "$OUT/pkg"
echo "sanitizer runs passed"
