// Host export of the transforms' LDS layouts (test infrastructure only), for
// the bank-conflict model checks.
#include <hip/hip_runtime.h>

#include "../../paper_1804_05335_amd/csrc/fdas_fft.hpp"

extern "C" int emu_lds_pad(int idx, int pair)
{
    return pair ? fdas::lds_pad<true>(idx) : fdas::lds_pad<false>(idx);
}
extern "C" int emu_pair_writes(int L)
{
    switch (L) {
    case 256:  return fdas::PairWrites<256>::value;
    case 512:  return fdas::PairWrites<512>::value;
    case 1024: return fdas::PairWrites<1024>::value;
    case 2048: return fdas::PairWrites<2048>::value;
    case 4096: return fdas::PairWrites<4096>::value;
    case 8192: return fdas::PairWrites<8192>::value;
    default:   return -1;
    }
}
