#!/bin/bash
# Host code (plan building, workspace sizing, validation) under AddressSanitizer and
# UndefinedBehaviorSanitizer, on the inputs of seven workloads.  CPU only.
set -euo pipefail
HERE="$(cd "$(dirname "$0")" && pwd)"
C="$HERE/../../paper_2006_10487_amd/csrc"
OUT="$(mktemp -d)"
python3 "$HERE/dump_inputs.py" "$OUT"
/opt/rocm/bin/hipcc -std=c++17 -O1 -g -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
    -Xclang -target-feature -Xclang -packed-fp32-ops --offload-arch=gfx950 -I"$C" \
    "$HERE/plan_main.cpp" "$C/prep.cpp" "$C/capi.cpp" "$C/adjoint.cpp" "$C/kernels.hip" -o "$OUT/plan_asan"
ASAN_OPTIONS=detect_leaks=1:halt_on_error=1 UBSAN_OPTIONS=halt_on_error=1 "$OUT/plan_asan" "$OUT"/*.bin
rm -rf "$OUT"
