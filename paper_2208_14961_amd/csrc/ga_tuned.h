// ga_tuned.h -- lanes per child of the children kernel, per order and
// launch size, as chosen by paper_2208_14961_amd/tune.py on one MI355X
// (mean generation time of a plain-GA run, binary tournament, SQ key; the
// times of every variant are in the comments).  Row i is order 4(i+1);
// entry j applies up to kTuneMaxChildren[j] children.  Regenerate with
// `python -m paper_2208_14961_amd.tune` on the GPU, then rebuild.
#pragma once
#include <stdint.h>

namespace ga {

constexpr int kTuneSizes = 5;
constexpr uint64_t kTuneMaxChildren[kTuneSizes] = {2048, 8192, 32768, 131072, ~0ull};
constexpr uint8_t kTunedLanes[16][kTuneSizes] = {
  {4, 4, 2, 2, 2},  // m = 4: n=1024: L2 3.1us L4 3.0us L8 3.1us; n=4096: L2 3.1us L4 3.1us L8 3.3us; n=16384: L2 3.4us L4 3.5us L8 3.6us; n=65536: L2 4.9us L4 5.0us L8 6.2us; n=262144: L2 8.8us L4 9.2us L8 12.2us
  {4, 4, 4, 4, 2},  // m = 8: n=1024: L2 3.2us L4 3.1us L8 3.1us; n=4096: L2 3.3us L4 3.2us L8 3.3us; n=16384: L2 3.8us L4 3.7us L8 3.8us; n=65536: L2 5.9us L4 5.8us L8 7.0us; n=262144: L2 9.9us L4 10.4us L8 13.0us
  {4, 4, 4, 4, 2},  // m = 12: n=1024: L2 3.5us L4 3.2us L8 3.2us; n=4096: L2 3.6us L4 3.4us L8 3.5us; n=16384: L2 4.3us L4 4.0us L8 4.2us; n=65536: L2 7.2us L4 7.0us L8 7.9us; n=262144: L2 12.4us L4 12.7us L8 14.9us
  {8, 4, 4, 4, 2},  // m = 16: n=1024: L2 3.7us L4 3.3us L8 3.3us; n=4096: L2 3.8us L4 3.4us L8 3.5us; n=16384: L2 4.6us L4 4.2us L8 4.2us; n=65536: L2 7.7us L4 7.2us L8 8.4us; n=262144: L2 12.9us L4 13.3us L8 15.7us
  {8, 8, 8, 4, 2},  // m = 20: n=1024: L2 3.9us L4 3.5us L8 3.4us; n=4096: L2 4.1us L4 3.7us L8 3.7us; n=16384: L2 5.1us L4 4.8us L8 4.7us; n=65536: L2 9.2us L4 9.0us L8 9.6us; n=262144: L2 16.0us L4 17.2us L8 18.8us
  {8, 8, 8, 4, 2},  // m = 24: n=1024: L2 4.3us L4 3.8us L8 3.5us; n=4096: L2 4.5us L4 4.0us L8 3.8us; n=16384: L2 5.5us L4 5.2us L8 5.1us; n=65536: L2 10.3us L4 10.1us L8 11.0us; n=262144: L2 17.4us L4 19.8us L8 23.8us
  {8, 8, 8, 4, 2},  // m = 28: n=1024: L2 4.6us L4 3.9us L8 3.6us; n=4096: L2 4.8us L4 4.1us L8 3.9us; n=16384: L2 6.1us L4 5.4us L8 5.4us; n=65536: L2 11.4us L4 10.9us L8 11.4us; n=262144: L2 20.7us L4 21.9us L8 24.4us
  {8, 8, 8, 4, 4},  // m = 32: n=1024: L2 5.1us L4 4.1us L8 3.7us; n=4096: L2 5.3us L4 4.2us L8 3.9us; n=16384: L2 6.3us L4 5.3us L8 5.1us; n=65536: L2 11.9us L4 10.3us L8 11.0us; n=262144: L2 24.6us L4 22.2us L8 24.5us
  {8, 8, 8, 4, 4},  // m = 36: n=1024: L4 5.7us L8 4.6us; n=4096: L4 6.1us L8 5.4us; n=16384: L4 8.4us L8 8.0us; n=65536: L4 16.3us L8 16.7us; n=262144: L4 44.3us L8 48.1us
  {8, 8, 4, 4, 4},  // m = 40: n=1024: L4 6.2us L8 4.9us; n=4096: L4 6.7us L8 5.7us; n=16384: L4 8.8us L8 8.8us; n=65536: L4 18.1us L8 19.1us; n=262144: L4 52.6us L8 58.7us
  {8, 8, 8, 4, 4},  // m = 44: n=1024: L4 6.7us L8 5.1us; n=4096: L4 7.2us L8 6.0us; n=16384: L4 10.0us L8 9.5us; n=65536: L4 19.9us L8 20.4us; n=262144: L4 58.6us L8 64.1us
  {8, 8, 8, 4, 4},  // m = 48: n=1024: L4 7.3us L8 5.3us; n=4096: L4 7.8us L8 6.1us; n=16384: L4 10.2us L8 9.7us; n=65536: L4 21.2us L8 21.3us; n=262144: L4 61.8us L8 67.2us
  {8, 8, 8, 4, 4},  // m = 52: n=1024: L4 7.9us L8 6.0us; n=4096: L4 8.5us L8 6.9us; n=16384: L4 11.7us L8 11.3us; n=65536: L4 24.6us L8 25.4us; n=262144: L4 76.0us L8 82.5us
  {8, 8, 8, 8, 4},  // m = 56: n=1024: L4 8.4us L8 6.1us; n=4096: L4 9.1us L8 7.1us; n=16384: L4 12.2us L8 11.6us; n=65536: L4 26.9us L8 26.4us; n=262144: L4 85.7us L8 86.5us
  {8, 8, 8, 8, 4},  // m = 60: n=1024: L4 9.3us L8 6.6us; n=4096: L4 9.9us L8 7.7us; n=16384: L4 13.6us L8 13.0us; n=65536: L4 30.5us L8 30.2us; n=262144: L4 95.8us L8 101.4us
  {8, 8, 8, 4, 4},  // m = 64: n=1024: L4 10.2us L8 7.1us; n=4096: L4 10.8us L8 8.0us; n=16384: L4 14.8us L8 14.0us; n=65536: L4 33.1us L8 34.3us; n=262144: L4 109.6us L8 119.1us
};

}  // namespace ga
