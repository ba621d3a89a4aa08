// The 3D sweeps (k_sweep<3, J>), in a translation unit of their own so that
// they can be compiled with the instruction scheduling that suits them (the
// build gives this file the scheduler's ILP-first strategy: 3D sweeps measured
// about 1 % faster with it, 2D ones 8 % slower).
#include "pa_sweep.h"

hipError_t pa_sweep3_launch(const PaRunDesc *runs, const PaBlk *map, int nblocks, int threads, size_t lds,
                            hipStream_t st, bool J, int theta, uint32_t t0, int gather)
{
    if (J)
        k_sweep<3, true><<<nblocks, threads, lds, st>>>(runs, map, theta, t0, gather);
    else
        k_sweep<3, false><<<nblocks, threads, lds, st>>>(runs, map, theta, t0, gather);
    return hipGetLastError();
}
