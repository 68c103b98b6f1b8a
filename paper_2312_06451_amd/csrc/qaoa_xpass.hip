// Tile passes of the X-product mixers (Sec. 2.1, Eq. (2)): a mixer made of products of X is
// diagonal after a basis change on every qubit. Eq. (2) writes it with Hadamards; here the
// change is V = R_y(pi/2) on every qubit (R_y(pi/2) Z R_y(pi/2)^dag = X as well), because in tan
// form R_y(+-pi/2) is I -+ i Y up to the scalar cos(pi/4): the pass kernel of the
// transverse-field path with Y butterflies (tau = +-1, four FMAs per amplitude pair, passengers
// at tau = 0) and the same scalar tracking. A layer is cost diagonal, V^dag, mixer diagonal, V;
// with the tile order alternating between transforms, the last tile of one transform and the
// first of the next share one pass with the diagonal between them.
#include <hip/hip_runtime.h>

#include "qaoa_internal.h"
#include "qaoa_tile.h"

namespace qaoa {

namespace {

template <typename R, int T, int KIND, typename TT, int SX>
hipError_t hpass_shape(const PassArgs<R> &a, int shape, int mixd, hipStream_t s) {
  if constexpr (KIND == 3) return launch_pass_t<R, T, 3, SX, SX, 1, TT, 1>(a, s);
  else {
    if (shape == 0) return launch_pass_t<R, T, KIND, SX, 0, 0, TT, 1>(a, s);
    if constexpr (KIND == 1)
      if (shape == 2) return launch_pass_t<R, T, 1, 0, SX, 2, TT, 1>(a, s);
    if (shape == 3) return launch_pass_t<R, T, KIND, SX, 0, 3, TT, 1>(a, s);
    if (shape == 1) {
      if (mixd == XD_POPCOUNT) return launch_pass_t<R, T, KIND, SX, SX, 1, TT, 2>(a, s);
      if (mixd == XD_TERMS) return launch_pass_t<R, T, KIND, SX, SX, 1, TT, 3>(a, s);
      if (mixd == XD_QUBIT) return launch_pass_t<R, T, KIND, SX, SX, 1, TT, 4>(a, s);
      if (mixd != 0) return hipErrorInvalidValue;
      return launch_pass_t<R, T, KIND, SX, SX, 1, TT, 1>(a, s);
    }
    return hipErrorInvalidValue;
  }
}

template <typename R, int T, int KIND, typename TT>
hipError_t hpass_sx(const PassArgs<R> &a, int sx, int shape, int mixd, hipStream_t s) {
  if (sx == 7) return hpass_shape<R, T, KIND, TT, 7>(a, shape, mixd, s);
  if (sx == 5) return hpass_shape<R, T, KIND, TT, 5>(a, shape, mixd, s);
  if (sx == 3) return hpass_shape<R, T, KIND, TT, 3>(a, shape, mixd, s);
  if (sx == 1) return hpass_shape<R, T, KIND, TT, 1>(a, shape, mixd, s);
  return hipErrorInvalidValue;
}

template <typename R, int T, typename TT>
hipError_t hpass_kind(const PassArgs<R> &a, int kind, int sx, int shape, int mixd, hipStream_t s) {
  if (kind == 1) return hpass_sx<R, T, 1, TT>(a, sx, shape, mixd, s);
  if (kind == 2) return hpass_sx<R, T, 2, TT>(a, sx, shape, mixd, s);
  if (kind == 3) return hpass_sx<R, T, 3, TT>(a, sx, shape, mixd, s);
  if (kind == 4) return hpass_sx<R, T, 4, TT>(a, sx, shape, mixd, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_hpass_f32(const PassArgs<float> &a, int kind, int sx, int shape, int tbytes, int mixd,
                           hipStream_t s) {
  return tbytes == 1 ? hpass_kind<float, TILE_BITS_F32, uint8_t>(a, kind, sx, shape, mixd, s)
                     : hpass_kind<float, TILE_BITS_F32, uint16_t>(a, kind, sx, shape, mixd, s);
}

hipError_t launch_hpass_f64(const PassArgs<double> &a, int kind, int sx, int shape, int tbytes, int mixd,
                           hipStream_t s) {
  return tbytes == 1 ? hpass_kind<double, TILE_BITS_F64, uint8_t>(a, kind, sx, shape, mixd, s)
                     : hpass_kind<double, TILE_BITS_F64, uint16_t>(a, kind, sx, shape, mixd, s);
}

}  // namespace qaoa
