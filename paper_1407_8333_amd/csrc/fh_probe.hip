// Microbenchmark of the LDS atomic rate of a gfx950 CU: the roof of the
// frequency-Hough tile kernel, whose every cell update is one ds_add_u32 with
// no return value.  Built as its own library (libfh_probe.so) and used only
// by the benchmark.
//
// One workgroup of 1024 threads per CU (128 KB of LDS each, so no second
// workgroup fits a CU).  Every lane holds 8 LDS word addresses computed
// before the timed loop, so the loop issues ds_add_u32 back to back with no
// address arithmetic.  Address patterns:
//   0  conflict free: a wave's 64 lanes hit 64 consecutive words
//   1  random words (a lane's 8 addresses drawn from a hash)
//   2  the tile kernel's pattern: each 16-lane group hits 16 consecutive
//      words (one column of 16 rows) at a column drawn from a hash, so the
//      four groups of a wave collide on banks as the real tiles do
//   3  one bank: every lane of a wave hits a different word of the same bank
//   4  the tile pattern with one column per group for all 8 atomics of a
//      round, so consecutive atomics of a lane hit the same word (as the
//      updates of out-of-tile stripes do in the tiles' dump columns)
//   5  the tile pattern with slanted stripes: lane j of a group hits column
//      c + floor(j s / 8) with a slope s in [-40, 40] / 8 columns per row
//      drawn per group, as a stripe crosses the 16 rows of a tile
//   6  the tile pattern with only lanes 0-2 of each group active (a row
//      block with 3 rows on the grid): 12 of 64 lanes per atomic, to show
//      whether the pipe's cost follows the active lanes or the instructions
//   7  the tile pattern with ds_add_f32 (floating-point accumulation)
// Cycles come from the shader clock (clock64) around the loop, between two
// workgroup barriers, and the same interval on the constant 100 MHz clock
// (wall_clock64) gives the shader clock's frequency under this load; the
// chip-wide rate comes from HIP events around the launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 1024;
constexpr int kWords = 32768;  // 128 KB
constexpr int kAddr = 8;

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    // integer finaliser (xorshift-multiply), any well-mixed hash serves
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(kThreads) k_lds_atomic(int32_t mode, int32_t iters, uint32_t seed,
                                                         unsigned long long *__restrict__ cycles,
                                                         unsigned long long *__restrict__ ticks,
                                                         uint32_t *__restrict__ sink) {
    __shared__ uint32_t lds[kWords];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < kWords; i += kThreads) lds[i] = 0;
    uint32_t a[kAddr];
#pragma unroll
    for (int k = 0; k < kAddr; ++k) {
        uint32_t w;
        if (mode == 0) {
            w = (uint32_t)((wave * kAddr + k) * 64 + lane);
        } else if (mode == 1) {
            w = hash32(seed ^ (uint32_t)(blockIdx.x * kThreads + tid) * 8u ^ (uint32_t)k * 0x9E3779B9u);
        } else if (mode == 5) {
            const uint32_t hh = hash32(seed ^ (uint32_t)(blockIdx.x * 64 + wave * 4 + (lane >> 4)) * 8u ^
                                       (uint32_t)k * 0x9E3779B9u);
            const int slope8 = (int)(hh >> 16) % 81 - 40;
            const int col = (int)(hh % 1024u) + 512 + ((lane & 15) * slope8 >> 3);
            w = (uint32_t)col * 16u + (uint32_t)(lane & 15);
        } else if (mode == 2 || mode == 4 || mode == 6 || mode == 7) {
            const uint32_t kk = mode == 4 ? 0u : (uint32_t)k;
            const uint32_t col = hash32(seed ^ (uint32_t)(blockIdx.x * 64 + wave * 4 + (lane >> 4)) * 8u ^
                                        kk * 0x9E3779B9u) % 2048u;
            w = col * 16u + (uint32_t)(lane & 15);
        } else {
            w = (uint32_t)lane * 32u + (uint32_t)(wave * kAddr + k) * 2048u;
        }
        a[k] = w & (kWords - 1);
    }
    const bool on = mode != 6 || (lane & 15) < 3;
    __syncthreads();
    const unsigned long long w0 = wall_clock64();
    const unsigned long long t0 = clock64();
    if (mode == 7) {
        float *fl = reinterpret_cast<float *>(lds);
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kAddr; ++k) atomicAdd(&fl[a[k]], 1.0f);
        }
    } else if (on) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kAddr; ++k) atomicAdd(&lds[a[k]], 1u);
        }
    }
    __syncthreads();
    const unsigned long long t1 = clock64();
    const unsigned long long w1 = wall_clock64();
    if (tid == 0) {
        cycles[blockIdx.x] = t1 - t0;
        ticks[blockIdx.x] = w1 - w0;
    }
    // keep the updates live: every word's count goes to memory
    for (int i = tid; i < kWords; i += kThreads) atomicAdd(sink + (i & 1023), lds[i]);
}

}  // namespace

extern "C" {

// Run pattern `mode` (0-7) with `blocks` workgroups of 1024 threads, each
// active lane issuing 8 * iters atomics.  Outputs: chip-wide lane-ops per
// second (HIP events around the launch), mean LDS atomic lanes (active ones)
// per shader clock per workgroup (clock64 around the loop), the launch time
// in ms, and the mean
// shader clock in GHz over the loops (clock64 cycles per wall_clock64 tick
// times 100 MHz).  Returns 0, or a HIP error code.
int fhp_lds_atomic(int32_t mode, int32_t iters, int32_t blocks, double *lane_ops_per_s,
                   double *lanes_per_clk, double *ms_out, double *clock_ghz) {
    if (mode < 0 || mode > 7 || iters < 1 || blocks < 1) return (int)hipErrorInvalidValue;
    unsigned long long *cyc = nullptr, *tck = nullptr;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&cyc, sizeof(unsigned long long) * (size_t)blocks);
    if (e == hipSuccess) e = hipMalloc(&tck, sizeof(unsigned long long) * (size_t)blocks);
    if (e == hipSuccess) e = hipMalloc(&sink, 4 * 1024);
    if (e == hipSuccess) e = hipMemset(sink, 0, 4 * 1024);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // one untimed launch first (code load, clocks ramping up)
    if (e == hipSuccess) {
        k_lds_atomic<<<blocks, kThreads>>>(mode, iters, 12345u, cyc, tck, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) {
        k_lds_atomic<<<blocks, kThreads>>>(mode, iters, 67890u, cyc, tck, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) {
        unsigned long long *h = new unsigned long long[blocks];
        unsigned long long *w = new unsigned long long[blocks];
        e = hipMemcpy(h, cyc, sizeof(unsigned long long) * (size_t)blocks, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(w, tck, sizeof(unsigned long long) * (size_t)blocks, hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            const double lanes = (double)kThreads * kAddr * (double)iters * (mode == 6 ? 3.0 / 16.0 : 1.0);
            double sum = 0.0, cyc_sum = 0.0, tick_sum = 0.0;
            for (int b = 0; b < blocks; ++b) {
                sum += lanes / (double)(h[b] ? h[b] : 1);
                cyc_sum += (double)h[b];
                tick_sum += (double)w[b];
            }
            *lanes_per_clk = sum / blocks;
            *lane_ops_per_s = lanes * blocks / (ms * 1e-3);
            *ms_out = ms;
            *clock_ghz = tick_sum > 0 ? cyc_sum / tick_sum * 0.1 : 0.0;
        }
        delete[] h;
        delete[] w;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (cyc) (void)hipFree(cyc);
    if (tck) (void)hipFree(tck);
    if (sink) (void)hipFree(sink);
    return (int)e;
}

}  // extern "C"
