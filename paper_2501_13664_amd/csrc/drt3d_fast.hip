// Shape-specialised DRT pass kernels of one (KX, KY) pass shape, compiled
// once per shape with -DDRT3D_KX=.. -DDRT3D_KY=.. so the shapes build in
// parallel.

#include "drt3d_kernels.h"

#if !defined(DRT3D_KX) || !defined(DRT3D_KY)
#error "compile with -DDRT3D_KX=<2|3> -DDRT3D_KY=<2|3>"
#endif

#define DRT3D_CAT2(a, b, c) a##b##_##c
#define DRT3D_CAT(a, b, c) DRT3D_CAT2(a, b, c)

namespace drt3d {

// 64-column groups (3.3) also come with 16 wavefronts per work group
constexpr bool kWide = DRT3D_KX == 3 && DRT3D_KY == 3;

template <typename T, int MODE, int NW>
static const void* mode_kernel(int nch)
{
#define DRT3D_NC(NC) \
    if (nch == NC) return reinterpret_cast<const void*>(&fast::drt_pass_fast<T, DRT3D_KX, DRT3D_KY, NC, MODE, NW>);
    DRT3D_NC(1) DRT3D_NC(2) DRT3D_NC(3) DRT3D_NC(4) DRT3D_NC(5) DRT3D_NC(6)
#undef DRT3D_NC
    return nullptr;
}

template <typename T, int NW>
static const void* shape_kernel(int nch, int mode)
{
    switch (mode) {
    case 0: return mode_kernel<T, 0, NW>(nch);
    case 1: return mode_kernel<T, 1, NW>(nch);
    case 2: return mode_kernel<T, 2, NW>(nch);
    default: return nullptr;
    }
}

// Narrow storage (uint32 arithmetic, eight wavefronts): source and destination
// bytes per element (sb, db) in {(1, 2), (2, 4), (1, 4)}, forward modes only.
template <int MODE, int SB, int DB>
static const void* narrow_kernel(int nch)
{
#define DRT3D_NC(NC)                                                                                        \
    if (nch == NC)                                                                                          \
        return reinterpret_cast<const void*>(&fast::drt_pass_fast<uint32_t, DRT3D_KX, DRT3D_KY, NC, MODE, 8, SB, DB>);
    DRT3D_NC(1) DRT3D_NC(2) DRT3D_NC(3) DRT3D_NC(4) DRT3D_NC(5) DRT3D_NC(6)
#undef DRT3D_NC
    return nullptr;
}

const void* DRT3D_CAT(drt_fast_kernel_narrow_, DRT3D_KX, DRT3D_KY)(int nch, int mode, int sb, int db)
{
    if (sb == 1 && db == 2 && mode == 0) return narrow_kernel<0, 1, 2>(nch);
    if (sb == 2 && db == 4 && mode == 0) return narrow_kernel<0, 2, 4>(nch);
    if (sb == 2 && db == 4 && mode == 1) return narrow_kernel<1, 2, 4>(nch);
    if (sb == 1 && db == 4 && mode == 1) return narrow_kernel<1, 1, 4>(nch);
    return nullptr;
}

#if DRT3D_KX == DRT3D_KY
// The adjoint's last pass fused over each volume layout group (square shapes).
template <typename T, int NW>
static const void* adj_group_nw(int nch)
{
#define DRT3D_NC(NC) \
    if (nch == NC) return reinterpret_cast<const void*>(&fast::drt_adj_last_group<T, DRT3D_KX, NC, NW>);
    DRT3D_NC(1) DRT3D_NC(2) DRT3D_NC(3) DRT3D_NC(4) DRT3D_NC(5) DRT3D_NC(6)
#undef DRT3D_NC
    return nullptr;
}

const void* DRT3D_CAT(drt_adj_group_kernel_, DRT3D_KX, DRT3D_KY)(int is_float, int nch, int waves)
{
    if (waves == 8) return is_float ? adj_group_nw<float, 8>(nch) : adj_group_nw<uint32_t, 8>(nch);
    if (kWide && waves == 16)
        return is_float ? adj_group_nw<float, kWide ? 16 : 8>(nch) : adj_group_nw<uint32_t, kWide ? 16 : 8>(nch);
    return nullptr;
}
#endif

// mode: 0 forward into a stage buffer, 1 the forward's last pass, 2 adjoint;
// waves: 8, or 16 for the 3.3 shape
const void* DRT3D_CAT(drt_fast_kernel_, DRT3D_KX, DRT3D_KY)(int is_float, int nch, int mode, int waves)
{
    if (waves == 8) return is_float ? shape_kernel<float, 8>(nch, mode) : shape_kernel<uint32_t, 8>(nch, mode);
    if (kWide && waves == 16)
        return is_float ? shape_kernel<float, kWide ? 16 : 8>(nch, mode)
                        : shape_kernel<uint32_t, kWide ? 16 : 8>(nch, mode);
    return nullptr;
}

}  // namespace drt3d
