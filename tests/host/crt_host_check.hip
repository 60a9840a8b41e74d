// Host build of the modular form's residue and reconstruction functions (split_tile.h), for a
// CPU test: the device-only qualifier is widened to host + device before the header is read.
// Reads lines "X g_0 .. g_15" (X a signed integer of up to 126 bits in decimal, g_k int32 with
// g_k = X mod p_k, then y, an integer of at most 53 significant bits with |y| < 2^62) and prints,
// per line, crt_reconstruct(g) as a hex float and the balanced residues of y from
// crt_residues_of((double) y), the FP64 residue routine of the residue kernels.
#include <hip/hip_runtime.h>
#undef __device__
#define __device__ __attribute__((host)) __attribute__((device))
#include "split_tile.h"

#include <cstdio>
#include <cstring>

using namespace zk;

int main() {
    char xs[64];
    while (scanf("%63s", xs) == 1) {
        int g[kCrtMods];
        for (int k = 0; k < kCrtMods; ++k)
            if (scanf("%d", &g[k]) != 1) return 2;
        long long y;
        if (scanf("%lld", &y) != 1) return 2;
        int d[kCrtMods];
        crt_residues_of((double)y, d);
        printf("%a", crt_reconstruct(g));
        for (int k = 0; k < kCrtMods; ++k) printf(" %d", d[k]);
        printf("\n");
    }
    return 0;
}
