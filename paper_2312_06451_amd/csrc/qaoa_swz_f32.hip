// Tile passes of the transverse-field mixer in the swizzled state layout (narrow covers: the top
// ten index bits folded into ten middle ones), float state. One access form per instantiation:
// XOR form with non-temporal (1) or cached (2) accesses, or the add form (3) for tiles whose own
// address bits all lie below the folded ones.
#include <hip/hip_runtime.h>

#include "qaoa_internal.h"
#include "qaoa_tile.h"

namespace qaoa {

namespace {

template <typename TT, int LAY>
hipError_t swz_kind(const PassArgs<float> &a, int kind, int shape, hipStream_t s) {
  if (kind == 1) return launch_shape<float, TILE_BITS_F32, 1, TT, 7, LAY>(a, shape, s);
  if (kind == 2) return launch_shape<float, TILE_BITS_F32, 2, TT, 7, LAY>(a, shape, s);
  if (kind == 4) return launch_shape<float, TILE_BITS_F32, 4, TT, 7, LAY>(a, shape, s);
  return launch_shape<float, TILE_BITS_F32, 3, TT, 7, LAY>(a, shape, s);
}

template <typename TT>
hipError_t swz_form(const PassArgs<float> &a, int kind, int shape, hipStream_t s) {
  if (a.cached) return swz_kind<TT, 2>(a, kind, shape, s);
  if (a.swz_add) return swz_kind<TT, 3>(a, kind, shape, s);
  return swz_kind<TT, 1>(a, kind, shape, s);
}

}  // namespace

hipError_t launch_pass_swz_f32(const PassArgs<float> &a, int kind, int sx, int shape, int tbytes,
                               hipStream_t s) {
  // the layout's instantiations cover the narrow covers' passes only
  if (sx != 7 || (a.flags & PF_LOAD_PSI0) || a.swz <= 0 || a.swz + 10 > a.swz_src) return hipErrorInvalidValue;
  return tbytes == 1 ? swz_form<uint8_t>(a, kind, shape, s) : swz_form<uint16_t>(a, kind, shape, s);
}

}  // namespace qaoa
