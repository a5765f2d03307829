// Instantiations of the transform passes, one group of lattice sizes per
// compilation (the build compiles this file once per QF_GROUP value).
#include "fft_passes.h"

namespace qf {

#if QF_GROUP == 0
void register_fft_group0(FftKernels *t) {
  register_size<8>(t); register_size<10>(t); register_size<12>(t); register_size<16>(t);
  register_size<18>(t); register_size<20>(t); register_size<24>(t); register_size<30>(t);
  register_size<32>(t);
}
#elif QF_GROUP == 1
void register_fft_group1(FftKernels *t) {
  register_size<36>(t); register_size<40>(t); register_size<48>(t); register_size<50>(t);
  register_size<54>(t); register_size<60>(t); register_size<64>(t); register_size<72>(t);
  register_size<80>(t);
}
#elif QF_GROUP == 2
void register_fft_group2(FftKernels *t) {
  register_size<90>(t); register_size<96>(t); register_size<100>(t); register_size<108>(t);
  register_size<120>(t); register_size<128>(t);
}
#elif QF_GROUP == 3
void register_fft_group3(FftKernels *t) {
  register_size<144>(t); register_size<150>(t); register_size<160>(t); register_size<162>(t);
  register_size<180>(t);
}
#else
void register_fft_group4(FftKernels *t) {
  register_size<192>(t); register_size<200>(t); register_size<216>(t); register_size<240>(t);
  register_size<250>(t); register_size<256>(t);
}
#endif

}  // namespace qf
