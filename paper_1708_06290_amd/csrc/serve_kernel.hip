// Work-item kernel of the serving layer: one launch runs shifts of different
// resident systems, with different n and m, drawn from a device work list.
//
// Every workgroup is one wavefront that repeatedly claims the next work item
// with an atomic counter and runs, for that shift, the FP64 sweep (the same
// device body as the batch kernel, so a shift gives identical results alone
// or in a mix) followed by its Q* pass.  The counter only grows, so every
// wave leaves the loop once the list is exhausted.
#include "serve.hpp"

namespace shs {

namespace {

template <int M>
constexpr int lds_need() { return sweep_lds_elems<double, M, false>(); }

template <int... Ms>
constexpr int max_lds(std::integer_sequence<int, Ms...>)
{
    int mx = 0;
    ((mx = lds_need<Ms + 1>() > mx ? lds_need<Ms + 1>() : mx), ...);
    return mx;
}

constexpr int kServeLds = max_lds(std::make_integer_sequence<int, 16>{});

// Each m is a separate function (not inlined) so that its registers are
// allocated as in the batch kernel of the same m; LDS is the launch's
// dynamic shared memory, sized for the largest m.
extern __shared__ double serve_lds[];

template <int M>
__device__ __noinline__ void run_item(const ServeItem *wp)
{
    using Sh = SweepShape<double, M, false>;
    const ServeItem w = *wp;
    double *lds = serve_lds;
    SweepItem<double> it;
    it.n = w.n;
    it.H = w.H;
    it.ldh = w.ldh;
    it.sgr = w.sr;
    it.sgi = w.si;
    it.rf = w.refl;
    it.Y = w.Y;
    it.E = nullptr;
    it.Rtop = w.Rtop;
    it.status = w.status;
    sweep_body<double, M, false>(it, lds, lds + Sh::CH);
    // the sweep's reflector and Y stores complete before the Q* pass reads them
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const int lane = threadIdx.x;
    const int c = lane < M ? lane : 0;
    qstar_body<double, M, false>(w.n, lane < M, c, w.refl, Sh::TT, refl_tile_stride<double>(Sh::TT, Sh::S), Sh::S,
                                 w.Y, w.X + (int64_t)c * w.ldx * 2, 0, 1.0);
}

}  // namespace

__global__ __launch_bounds__(64, 2) void serve_kernel(const ServeItem *items, int count, unsigned *counter)
{
    __shared__ int claim;
    for (;;) {
        if (threadIdx.x == 0) claim = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int idx = claim;
        __syncthreads();
        if (idx >= count) return;
        const ServeItem *w = items + idx;
        switch (w->m) {
        case 1: run_item<1>(w); break;
        case 2: run_item<2>(w); break;
        case 3: run_item<3>(w); break;
        case 4: run_item<4>(w); break;
        case 5: run_item<5>(w); break;
        case 6: run_item<6>(w); break;
        case 7: run_item<7>(w); break;
        case 8: run_item<8>(w); break;
        case 9: run_item<9>(w); break;
        case 10: run_item<10>(w); break;
        case 11: run_item<11>(w); break;
        case 12: run_item<12>(w); break;
        case 13: run_item<13>(w); break;
        case 14: run_item<14>(w); break;
        case 15: run_item<15>(w); break;
        case 16: run_item<16>(w); break;
        default: break;
        }
        __syncthreads();
    }
}

int serve_max_waves() { return 2048; }

hipError_t launch_serve(const ServeItem *items, int count, unsigned *counter, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int grid = count < serve_max_waves() ? count : serve_max_waves();
    hipLaunchKernelGGL(serve_kernel, dim3(grid), dim3(kWave), sizeof(double) * kServeLds, st, items, count,
                       counter);
    return hipGetLastError();
}

}  // namespace shs
