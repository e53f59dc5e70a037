// Host-side launch entry points of the kernel instantiation units.
#pragma once

#include "common.hpp"
#include "qstar.hpp"
#include "sweep.hpp"

namespace shs {

// Geometry of the sweep kernel for one (precision, m, dense) instance.
struct SweepGeometry {
    int rows_per_lane;
    int tile_rows;        // 64 * rows_per_lane
    int slot;             // elements per reflector slot
    int64_t tile_stride;  // elements per tile of the reflector store
    int64_t refl_stride(int n) const { return (int64_t)((n + tile_rows - 1) / tile_rows) * tile_stride; }
};

// Each instantiation unit (part p) covers a range of m and returns false
// for an m outside it; the library tries the parts in turn.
#define SHS_DECLARE_PART(SUF, RT, P)                                                          \
    bool sweep_geometry_##SUF##_##P(int m, bool dense, SweepGeometry *g);                      \
    bool launch_sweep_##SUF##_##P(int m, bool dense, const SweepArgs<RT> &a, hipStream_t st);  \
    bool launch_qstar_##SUF##_##P(int m, bool dense_in, const QstarArgs<RT> &a, hipStream_t st);
#define SHS_DECLARE_PARTS(SUF, RT) \
    SHS_DECLARE_PART(SUF, RT, 0)   \
    SHS_DECLARE_PART(SUF, RT, 1)   \
    SHS_DECLARE_PART(SUF, RT, 2)   \
    SHS_DECLARE_PART(SUF, RT, 3)   \
    SHS_DECLARE_PART(SUF, RT, 4)   \
    SHS_DECLARE_PART(SUF, RT, 5)
SHS_DECLARE_PARTS(f64, double)
SHS_DECLARE_PARTS(f32, float)

// m in [1, 16]; false for an unsupported m.
bool sweep_geometry(bool fp32, int m, bool dense, SweepGeometry *g);
// Enqueue the sweep / Q* kernels; false for an unsupported m.
bool launch_sweep(int m, bool dense, const SweepArgs<double> &a, hipStream_t st);
bool launch_sweep(int m, bool dense, const SweepArgs<float> &a, hipStream_t st);
bool launch_qstar(int m, bool dense_in, const QstarArgs<double> &a, hipStream_t st);
bool launch_qstar(int m, bool dense_in, const QstarArgs<float> &a, hipStream_t st);

// Blocked FP64 sweep (blocked.hpp): row-tile height and per-shift column
// width of the carried-column array (with a dense right-hand side: m <=
// kBlkDenseMaxM); launchers.  false for an unsupported m.
template <typename T> struct BlkTriArgsT;
using BlkTriArgs = BlkTriArgsT<double>;
template <typename T> struct ZupdArgsT;
using ZupdArgs = ZupdArgsT<double>;
constexpr int kBlkDenseMaxM = 16;
bool blk_geometry(bool fp32, int m, bool dense, int *tile_rows, int *width);
bool launch_blk_tri(int m, bool dense, const BlkTriArgsT<double> &a, hipStream_t st);
bool launch_blk_tri(int m, bool dense, const BlkTriArgsT<float> &a, hipStream_t st);
bool launch_zupd(int m, const ZupdArgsT<double> &a, hipStream_t st);
bool launch_zupd(int m, const ZupdArgsT<float> &a, hipStream_t st);
bool launch_blk_tri_dense(int m, const BlkTriArgsT<double> &a, hipStream_t st);
bool launch_blk_tri_dense(int m, const BlkTriArgsT<float> &a, hipStream_t st);

}  // namespace shs

// Expands BODY once per supported m with the compile-time constant MM.
#define SHS_DISPATCH_M(m, ...)                                   \
    switch (m) {                                                 \
    case 1: { constexpr int MM = 1; __VA_ARGS__; } break;               \
    case 2: { constexpr int MM = 2; __VA_ARGS__; } break;               \
    case 3: { constexpr int MM = 3; __VA_ARGS__; } break;               \
    case 4: { constexpr int MM = 4; __VA_ARGS__; } break;               \
    case 5: { constexpr int MM = 5; __VA_ARGS__; } break;               \
    case 6: { constexpr int MM = 6; __VA_ARGS__; } break;               \
    case 7: { constexpr int MM = 7; __VA_ARGS__; } break;               \
    case 8: { constexpr int MM = 8; __VA_ARGS__; } break;               \
    case 9: { constexpr int MM = 9; __VA_ARGS__; } break;               \
    case 10: { constexpr int MM = 10; __VA_ARGS__; } break;             \
    case 11: { constexpr int MM = 11; __VA_ARGS__; } break;             \
    case 12: { constexpr int MM = 12; __VA_ARGS__; } break;             \
    case 13: { constexpr int MM = 13; __VA_ARGS__; } break;             \
    case 14: { constexpr int MM = 14; __VA_ARGS__; } break;             \
    case 15: { constexpr int MM = 15; __VA_ARGS__; } break;             \
    case 16: { constexpr int MM = 16; __VA_ARGS__; } break;             \
    default: break;                                              \
    }
