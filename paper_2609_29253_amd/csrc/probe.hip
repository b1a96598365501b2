// Vector-ALU peak of the device as the library's kernels are built (FP32 not
// packed): an FMA-only kernel with sixteen independent chains per lane, all
// operands in vector registers and no memory access in its loop, timed with
// HIP events.  On gfx950 an unpacked FP32 FMA issues at twice the FP64 rate.  The benchmark uses it to
// place the published peaks on the machine it runs on.
#include <hip/hip_runtime.h>

#include "patop.h"

namespace {

constexpr int kChains = 16;
constexpr int kProbeThreads = 256;
constexpr int kIters = 4096;

template <class T>
__global__ __launch_bounds__(kProbeThreads) void k_fma_peak(T* __restrict__ out, T b, T c, int iters)
{
    T x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = (T)(threadIdx.x + j) * (T)1e-3;
    // both multiplier and addend in vector registers (the empty statements only
    // pin them there): an FP32 FMA reading two scalar registers issues at about
    // two thirds of the rate of the all-vector form on gfx950
    T bv = b, cv = c;
    asm volatile("" : "+v"(bv));
    asm volatile("" : "+v"(cv));
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) x[j] = fma(x[j], bv, cv);
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += x[j];
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

template <class T>
hipError_t time_peak(int blocks, void* buf, double* flops)
{
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return e; }
    const T b = (T)0.999999, c = (T)1e-7;   // a contraction: the chains stay bounded
    k_fma_peak<T><<<blocks, kProbeThreads>>>((T*)buf, b, c, kIters / 8);   // warm-up
    (void)hipEventRecord(e0, nullptr);
    k_fma_peak<T><<<blocks, kProbeThreads>>>((T*)buf, b, c, kIters);
    (void)hipEventRecord(e1, nullptr);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) *flops = 2.0 * kChains * (double)kIters * kProbeThreads * blocks / (ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

extern "C" pat_status pat_probe_peak(int32_t device, double* out)
{
    if (!out) return PAT_E_ARG;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (hipSetDevice(device) != hipSuccess) return PAT_E_DEVICE;
    hipDeviceProp_t prop;
    pat_status st = PAT_OK;
    void* buf = nullptr;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        st = PAT_E_DEVICE;
    } else {
        const int blocks = 8 * prop.multiProcessorCount;
        if (hipMalloc(&buf, (size_t)blocks * kProbeThreads * sizeof(double)) != hipSuccess) {
            st = PAT_E_OOM;
        } else if (time_peak<double>(blocks, buf, &out[0]) != hipSuccess ||
                   time_peak<float>(blocks, buf, &out[1]) != hipSuccess) {
            st = PAT_E_DEVICE;
        }
        out[2] = prop.multiProcessorCount;
        out[3] = prop.clockRate * 1e-6;   // kHz -> GHz
    }
    if (buf) (void)hipFree(buf);
    (void)hipGetLastError();
    if (prev >= 0) (void)hipSetDevice(prev);
    return st;
}
