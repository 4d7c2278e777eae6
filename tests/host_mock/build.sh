#!/bin/bash
# Build the library's host code (every source compiled host-only, with
# AddressSanitizer and UndefinedBehaviorSanitizer), the CPU stand-in of the
# HIP runtime (mock_hip.cpp) and the entry-point driver of tests/host_asan
# into _build/mock/, with no GPU and no HIP runtime library.  Run from the
# repository root:
#   bash tests/host_mock/build.sh && _build/mock/driver
set -e
ROOT=$(pwd)
OUT=$ROOT/_build/mock
mkdir -p $OUT
SAN="-fsanitize=address,undefined -fno-omit-frame-pointer -fno-sanitize-recover=undefined"
for f in standardize syrk colsolve kkt polish output warm dense api; do
  /opt/rocm/bin/hipcc --cuda-host-only -O1 -g -std=c++17 -fPIC $SAN -I $ROOT/include \
    -c $ROOT/paper_2203_15031_amd/csrc/$f.hip -o $OUT/$f.o 2>&1 | grep -v "unused during compilation" || true &
done
/opt/rocm/llvm/bin/clang++ -O1 -g -std=c++17 -fPIC $SAN -I $ROOT/include \
  -c $ROOT/paper_2203_15031_amd/csrc/penalty.cpp -o $OUT/penalty.o &
/opt/rocm/llvm/bin/clang++ -O1 -g -std=c++17 -fPIC $SAN -D__HIP_PLATFORM_AMD__ -I /opt/rocm/include \
  -c $ROOT/tests/host_mock/mock_hip.cpp -o $OUT/mock_hip.o &
/opt/rocm/llvm/bin/clang++ -O1 -g -std=c++17 -fPIC $SAN -D__HIP_PLATFORM_AMD__ -I /opt/rocm/include -I $ROOT/include \
  -c $ROOT/tests/host_asan/driver.cpp -o $OUT/driver.o &
wait
for f in standardize syrk colsolve kkt polish output warm dense api; do
  [ -f $OUT/$f.o ] || { echo "compile of $f.hip failed"; exit 1; }
done
# the host-only objects name the device code objects they would register;
# there are none here
nm -u $OUT/*.o | awk '/__hip_fatbin_/ {print $2}' | sort -u | \
  awk '{printf "extern \"C\" const unsigned char %s[16] = {0};\n", $1}' > $OUT/fatbin_stubs.cpp
/opt/rocm/llvm/bin/clang++ -O1 -std=c++17 -fPIC -c $OUT/fatbin_stubs.cpp -o $OUT/fatbin_stubs.o
/opt/rocm/llvm/bin/clang++ $SAN $OUT/standardize.o $OUT/syrk.o $OUT/colsolve.o $OUT/kkt.o $OUT/polish.o \
  $OUT/output.o $OUT/warm.o $OUT/dense.o $OUT/api.o $OUT/penalty.o $OUT/mock_hip.o $OUT/fatbin_stubs.o \
  $OUT/driver.o -lpthread -o $OUT/driver
echo "built $OUT/driver"
/opt/rocm/llvm/bin/clang++ -O1 -g -std=c++17 $SAN -D__HIP_PLATFORM_AMD__ -I /opt/rocm/include \
  $ROOT/tests/host_mock/selftest.cpp $OUT/mock_hip.o -lpthread -o $OUT/selftest
echo "built $OUT/selftest"
