// single.hip -- functionals of one PCF at a time (paper, Section 3.2 "PCF
// integrals"): F(f) = r(int_a^b h(f(t)) dt) for every PCF of a set.
//
// Segment iteration (Algorithm IterateSegments) walks a PCF's pieces and
// adds (r - l) h(v) per segment [l, r) of [a, b). Piece k of a PCF is
// [t_k, t_{k+1}) (t_n = inf), so its segment is that piece clipped to
// [a, b); the segments of all pieces, summed, are the walk's segments. One
// wave per PCF: lane j takes pieces j, j + 64, ..., and the 64 partial sums
// are added by a fixed butterfly, so results do not depend on timing. With
// b = inf the unbounded last piece adds 0 when h(v_last) = 0 and an infinity
// of the sign of h(v_last) otherwise. The work is one pass over the set's
// rows: HBM-bound (16 B per FP64 row, 8 B per FP32 row, plus the offsets).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace pcf {

// h of the single-PCF kinds: SK_VALUE h(v) = v; SK_ABS |v|; SK_SQR v^2;
// SK_POW |v|^p.
enum { SK_VALUE = 0, SK_ABS = 1, SK_SQR = 2, SK_POW = 3 };

template <int SK>
__device__ __forceinline__ double h_single(double v, double p)
{
    if constexpr (SK == SK_VALUE)
        return v;
    else if constexpr (SK == SK_ABS)
        return fabs(v);
    else if constexpr (SK == SK_SQR)
        return v * v;
    else
        return pow(fabs(v), p);
}

// Sum over the 64 lanes of a wave by a butterfly of fixed shape.
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        x += __shfl_xor(x, o, 64);
    return x;
}

template <typename T, int SK>
__global__ void single_functional(SingleArgs a)
{
    const T *__restrict__ t = reinterpret_cast<const T *>(a.t);
    const T *__restrict__ v = reinterpret_cast<const T *>(a.v);
    T *__restrict__ out = reinterpret_cast<T *>(a.out);
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < a.n;
         i += nwaves) {
        const int64_t o0 = a.offsets[i], o1 = a.offsets[i + 1];
        double acc = 0.0;
        int tail = 0;  // sign of h on an unbounded last piece
        for (int64_t k = o0 + lane; k < o1; k += 64) {
            const double tk = (double)t[k];
            const double tn = k + 1 < o1 ? (double)t[k + 1] : INFINITY;
            const double l = tk > a.a ? tk : a.a;
            const double r = tn < a.b ? tn : a.b;
            if (r > l) {
                const double hv = h_single<SK>((double)v[k], a.p);
                if (r == INFINITY)
                    tail = hv > 0.0 ? 1 : (hv < 0.0 ? -1 : 0);
                else
                    acc += (r - l) * hv;
            }
        }
        acc = wave_sum(acc);
        // the tail is set on one lane at most (the last piece)
        int tl = tail;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            tl |= __shfl_xor(tl, o, 64);
        if (lane == 0) {
            double res = tl == 0 ? acc : (tl > 0 ? INFINITY : -INFINITY);
            if (a.root == 1)
                res = sqrt(res);
            else if (a.root == 2)
                res = pow(res, 1.0 / a.p);
            out[i] = (T)res;
        }
    }
}

template <typename T, int SK>
static hipError_t launch_single_t(const SingleArgs &a, hipStream_t s)
{
    int64_t blocks = (a.n + 3) / 4;  // 4 waves of 64 per block
    if (blocks > 8192)
        blocks = 8192;
    hipLaunchKernelGGL((single_functional<T, SK>), dim3((unsigned)blocks), dim3(256), 0,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_single(bool f64, int sk, const SingleArgs &a, hipStream_t s)
{
    if (a.n <= 0)
        return hipSuccess;
    if (f64) {
        switch (sk) {
        case SK_VALUE: return launch_single_t<double, SK_VALUE>(a, s);
        case SK_ABS: return launch_single_t<double, SK_ABS>(a, s);
        case SK_SQR: return launch_single_t<double, SK_SQR>(a, s);
        default: return launch_single_t<double, SK_POW>(a, s);
        }
    }
    switch (sk) {
    case SK_VALUE: return launch_single_t<float, SK_VALUE>(a, s);
    case SK_ABS: return launch_single_t<float, SK_ABS>(a, s);
    case SK_SQR: return launch_single_t<float, SK_SQR>(a, s);
    default: return launch_single_t<float, SK_POW>(a, s);
    }
}

}  // namespace pcf
