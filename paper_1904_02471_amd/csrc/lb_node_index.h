// lb_node_index.h -- row-major node index -> (x, y) by 32-bit division.  A
// grid holds at most 2^30 nodes (lb_create's limit), so the index fits an
// unsigned 32-bit integer and the 64-bit division, a long software sequence
// on the GPU, is not needed.
#pragma once

__device__ __forceinline__ void node_xy(long long n, int Nx, int &x, int &y)
{
    const unsigned u = (unsigned)n, w = (unsigned)Nx;
    const unsigned q = u / w;
    y = (int)q;
    x = (int)(u - q * w);
}
