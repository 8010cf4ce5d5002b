#!/bin/sh
# Builds the plain C oracle (test infrastructure only) into oracle/liborc.so.
set -e
here=$(cd "$(dirname "$0")" && pwd)
gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -fPIC -shared -std=c11 \
    -o "$here/liborc.so" "$here/native.c" -lm
