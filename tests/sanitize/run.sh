#!/bin/bash
# Host code under AddressSanitizer and UndefinedBehaviorSanitizer, CPU only: the library's
# plan building, workspace sizing and validation on the inputs of seven workloads, then the
# oracle's pin tests against a sanitized build of the oracle.
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
# the oracle is loaded by Python, so the sanitizer runtimes are preloaded into that process;
# never on top of another preload
if [ -n "${LD_PRELOAD:-}" ]; then echo "LD_PRELOAD is set; not running the oracle part" >&2; exit 1; fi
LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)" \
    ASAN_OPTIONS=detect_leaks=0:halt_on_error=1 OMP_NUM_THREADS=4 python3 "$HERE/oracle_sanitized.py"
