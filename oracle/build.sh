#!/bin/sh
# Builds the oracle shared library (test infrastructure only).
set -e
cd "$(dirname "$0")"
gcc -O2 -std=c11 -D_GNU_SOURCE -fPIC -shared -Wall -Wextra -Wno-unused-parameter \
    -ffp-contract=off -o liboracle.so refelem.c mesh.c dg.c chain.c -lm
