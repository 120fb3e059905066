#!/bin/bash
# Host-code sanitizer run of the library (AddressSanitizer + UndefinedBehaviorSanitizer on
# the host pass only; device code is built as usual).
#   tests/sanitize_runtime.sh build   compile _build/asan/libkc_asan.so and the driver
#                                      tests/sanitize_runtime.cpp (any machine with hipcc)
#   tests/sanitize_runtime.sh run     run the driver (needs the GPU); exit status = failures
set -euo pipefail
HERE="$(cd "$(dirname "$0")" && pwd)"
ROOT="$(dirname "$HERE")"
OUT="$ROOT/_build/asan"
ROCM="${ROCM_PATH:-/opt/rocm}"
case "${1:-}" in
  build)
    mkdir -p "$OUT"
    "$ROCM/bin/hipcc" --offload-arch=gfx950 -O2 -g -std=c++17 -shared -fPIC \
      -Xclang -target-feature -Xclang -packed-fp32-ops \
      -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all \
      -Xarch_host -fno-omit-frame-pointer \
      -o "$OUT/libkc_asan.so" "$ROOT/paper_2407_07718_amd/csrc/kc_api.hip"
    "$ROCM/llvm/bin/clang++" -O1 -g -std=c++17 -fopenmp -fsanitize=address,undefined -fno-sanitize-recover=all \
      -fno-omit-frame-pointer -D__HIP_PLATFORM_AMD__ -I"$ROCM/include" -I"$ROOT/include" \
      -o "$OUT/sanitize_runtime" "$HERE/sanitize_runtime.cpp" "$ROOT/oracle/kc_oracle.cpp" \
      -L"$OUT" -lkc_asan -L"$ROCM/lib" -lamdhip64 -Wl,-rpath,"$OUT" -Wl,-rpath,"$ROCM/lib" \
      -Wl,-rpath,"$ROCM/llvm/lib"
    ;;
  run)
    # leaks inside the HIP runtime's own allocations are not this library's
    printf 'leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\n' > "$OUT/lsan.supp"
    ASAN_OPTIONS="detect_leaks=1:protect_shadow_gap=0:halt_on_error=1" \
    LSAN_OPTIONS="suppressions=$OUT/lsan.supp" UBSAN_OPTIONS="print_stacktrace=1" \
      "$OUT/sanitize_runtime"
    ;;
  *)
    echo "usage: $0 build|run" >&2
    exit 2
    ;;
esac
