// Output tiles of the convolution body, shared by the host (piece counts)
// and the device (tile walk): 16 output pixels by 32 channels, or by 16
// channels when 32-channel tiles would give fewer than 128 tiles, so that a
// batch-1 layer spreads over more workgroups.
#pragma once
#include <stdint.h>

namespace acs {

constexpr int64_t kConvMinTiles = 128;

// Columns per tile for a layer of m output pixels (a multiple of 16) and
// cout output channels (a multiple of 32).
inline constexpr int32_t conv_tile_cols(int64_t m, int32_t cout)
{
    return (m / 16) * (cout / 32) >= kConvMinTiles ? 32 : 16;
}

inline constexpr int64_t conv_tiles(int64_t m, int32_t cout) { return (m / 16) * (cout / conv_tile_cols(m, cout)); }

}  // namespace acs
