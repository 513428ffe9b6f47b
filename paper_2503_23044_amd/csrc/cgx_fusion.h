// Launch declarations of the TSDF fusion's texel path (kept apart from
// cgx_common.h, whose contents the raster kernels depend on).
#pragma once
#include "cgx_common.h"

namespace cgx {

// depth and planar rgb of every view -> one float4 texel (d, r, g, b) per
// pixel, packed layout
void launch_tsdf_pack(int n_pixels, const float* depth, const float* rgb, const TsdfPack& cams,
                      int count, float4* texels, hipStream_t s);
// as launch_tsdf_integrate, gathering (d, r, g, b) texels
void launch_tsdf_integrate_texels(const TsdfPack& cams, int count, int nx, int ny, int n, double mu,
                                  const float4* texels, float* tsdf, float* weight, float* color,
                                  hipStream_t s);

}  // namespace cgx
