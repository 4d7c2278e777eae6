#!/bin/bash
# Build the library and tests/host_asan/driver.cpp with AddressSanitizer and
# UndefinedBehaviorSanitizer on the HOST code only (the device code objects
# are the ordinary ones), into _build/asan/.  Run from the repository root:
#   bash tests/host_asan/build.sh && ASAN_OPTIONS=detect_leaks=0:verify_asan_link_order=0 _build/asan/driver
set -e
ROOT=$(pwd)
OUT=$ROOT/_build/asan
mkdir -p $OUT
SAN="-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer"
for f in standardize syrk colsolve kkt polish output warm dense api; do
  /opt/rocm/bin/hipcc -O1 -g -std=c++17 -fPIC --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
    $SAN -I $ROOT/include -c $ROOT/paper_2203_15031_amd/csrc/$f.hip -o $OUT/$f.o &
done
/opt/rocm/llvm/bin/clang++ -O1 -g -std=c++17 -fPIC -fsanitize=address,undefined -I $ROOT/include \
  -c $ROOT/paper_2203_15031_amd/csrc/penalty.cpp -o $OUT/penalty.o &
wait
RT=$(/opt/rocm/llvm/bin/clang++ -print-resource-dir)/lib/linux
/opt/rocm/llvm/bin/clang++ -shared -fsanitize=address,undefined -shared-libsan $OUT/*.o -L/opt/rocm/lib -lamdhip64 \
  -Wl,-rpath,/opt/rocm/lib -Wl,-rpath,$RT -o $OUT/libspmesl_asan.so
/opt/rocm/llvm/bin/clang++ -O1 -g -std=c++17 -fsanitize=address,undefined -shared-libsan -D__HIP_PLATFORM_AMD__ \
  -I /opt/rocm/include -I $ROOT/include $ROOT/tests/host_asan/driver.cpp -L$OUT -lspmesl_asan -L/opt/rocm/lib -lamdhip64 \
  -Wl,-rpath,$OUT -Wl,-rpath,/opt/rocm/lib -Wl,-rpath,$RT -o $OUT/driver
echo "built $OUT/driver"
