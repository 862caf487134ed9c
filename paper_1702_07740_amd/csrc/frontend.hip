// Multi-dimensional reverse reconciliation front-end (Sec. II-C.3), gfx950.
//
// d-dimensional reconciliation, d in {1, 2, 4, 8}, groups the samples of a
// frame into d-tuples.  Bob sends M = U Y per tuple, U = ((-1)^{c_1}, ...,
// (-1)^{c_d}), Y = X + Z; Alice forms R = M X^{-1} = U + N.  The noise N is
// isotropic with per-coordinate variance d sigma^2 / |X|^2, so the channel LLR
// of coordinate i is
//     2 R_i |X|^2 / (d sigma^2) = 2 (M conj(X))_i / (d sigma^2),
// since X^{-1} = conj(X) / |X|^2.  The products are Cayley-Dickson products:
// an element of dimension 2k is a pair (a, b) of dimension-k elements and
//     (a, b)(c, e) = (a c - conj(e) b,  e a + b conj(c)),  conj(a, b) = (conj(a), -b),
// which gives the complex numbers, quaternions and octonions for d = 2, 4, 8.
//
// One thread per tuple; tuples are 4*d bytes, so loads and stores of a wave
// are contiguous.  Frames are padded to a whole number of tuples: the inputs
// hold n_d = d * ceil(n / d) samples, padding key bits are 0, and only the
// first n LLRs are written.
#include "internal.h"

namespace ldpc {

namespace {

constexpr int kBlock = 256;

template <int N>
struct CD {
    float v[N];
};

template <int N>
__device__ __forceinline__ CD<N> cd_conj(const CD<N> &x) {
    CD<N> r;
    r.v[0] = x.v[0];
#pragma unroll
    for (int i = 1; i < N; ++i) r.v[i] = -x.v[i];
    return r;
}

template <int N>
__device__ __forceinline__ CD<N / 2> half_lo(const CD<N> &x) {
    CD<N / 2> r;
#pragma unroll
    for (int i = 0; i < N / 2; ++i) r.v[i] = x.v[i];
    return r;
}

template <int N>
__device__ __forceinline__ CD<N / 2> half_hi(const CD<N> &x) {
    CD<N / 2> r;
#pragma unroll
    for (int i = 0; i < N / 2; ++i) r.v[i] = x.v[N / 2 + i];
    return r;
}

template <int N>
__device__ __forceinline__ CD<N> cd_mul(const CD<N> &x, const CD<N> &y);

template <>
__device__ __forceinline__ CD<1> cd_mul<1>(const CD<1> &x, const CD<1> &y) {
    CD<1> r;
    r.v[0] = x.v[0] * y.v[0];
    return r;
}

template <int N>
__device__ __forceinline__ CD<N> cd_mul(const CD<N> &x, const CD<N> &y) {
    const CD<N / 2> a = half_lo(x), b = half_hi(x), c = half_lo(y), e = half_hi(y);
    const CD<N / 2> ac = cd_mul(a, c), eb = cd_mul(cd_conj(e), b);
    const CD<N / 2> ea = cd_mul(e, a), bc = cd_mul(b, cd_conj(c));
    CD<N> r;
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
        r.v[i] = ac.v[i] - eb.v[i];
        r.v[N / 2 + i] = ea.v[i] + bc.v[i];
    }
    return r;
}

template <int Dm>
__device__ __forceinline__ CD<Dm> load_tuple(const float *p) {
    CD<Dm> r;
#pragma unroll
    for (int i = 0; i < Dm; ++i) r.v[i] = p[i];
    return r;
}

// Alice: LLR_i = 2 (M conj(X))_i / (d sigma^2) for the first n coordinates.
template <int Dm>
__global__ __launch_bounds__(kBlock) void llr_kernel(int n, int nd, const float *x,
                                                     const float *m, float scale, float *llr) {
    const int f = blockIdx.y;
    const int tup = blockIdx.x * kBlock + threadIdx.x;
    if (tup * Dm >= nd) return;
    const size_t base = (size_t)f * nd + (size_t)tup * Dm;
    const CD<Dm> X = load_tuple<Dm>(x + base);
    const CD<Dm> M = load_tuple<Dm>(m + base);
    const CD<Dm> P = cd_mul(M, cd_conj(X));
    float *out = llr + (size_t)f * n;
#pragma unroll
    for (int i = 0; i < Dm; ++i) {
        const int v = tup * Dm + i;
        if (v < n) out[v] = scale * P.v[i];
    }
}

// Bob: M = U Y with U_i = (-1)^{c_i}; padding coordinates (v >= n) take c = 0.
template <int Dm>
__global__ __launch_bounds__(kBlock) void message_kernel(int n, int nd, const uint8_t *bits,
                                                         const float *y, float *m) {
    const int f = blockIdx.y;
    const int tup = blockIdx.x * kBlock + threadIdx.x;
    if (tup * Dm >= nd) return;
    const size_t base = (size_t)f * nd + (size_t)tup * Dm;
    CD<Dm> U;
#pragma unroll
    for (int i = 0; i < Dm; ++i) {
        const int v = tup * Dm + i;
        const int c = v < n ? (bits[(size_t)f * n + v] & 1) : 0;
        U.v[i] = c ? -1.0f : 1.0f;
    }
    const CD<Dm> P = cd_mul(U, load_tuple<Dm>(y + base));
#pragma unroll
    for (int i = 0; i < Dm; ++i) m[base + i] = P.v[i];
}

}  // namespace

hipError_t enqueue_reconciliation_llr(int d, int F, int n, const float *x, const float *m,
                                      float sigma2, float *llr, hipStream_t st) {
    const int nd = d * ((n + d - 1) / d);
    const dim3 grid((unsigned)((nd / d + kBlock - 1) / kBlock), (unsigned)F);
    const float scale = 2.0f / ((float)d * sigma2);
    switch (d) {
        case 1: llr_kernel<1><<<grid, kBlock, 0, st>>>(n, nd, x, m, scale, llr); break;
        case 2: llr_kernel<2><<<grid, kBlock, 0, st>>>(n, nd, x, m, scale, llr); break;
        case 4: llr_kernel<4><<<grid, kBlock, 0, st>>>(n, nd, x, m, scale, llr); break;
        case 8: llr_kernel<8><<<grid, kBlock, 0, st>>>(n, nd, x, m, scale, llr); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t enqueue_reconciliation_message(int d, int F, int n, const uint8_t *bits, const float *y,
                                          float *m, hipStream_t st) {
    const int nd = d * ((n + d - 1) / d);
    const dim3 grid((unsigned)((nd / d + kBlock - 1) / kBlock), (unsigned)F);
    switch (d) {
        case 1: message_kernel<1><<<grid, kBlock, 0, st>>>(n, nd, bits, y, m); break;
        case 2: message_kernel<2><<<grid, kBlock, 0, st>>>(n, nd, bits, y, m); break;
        case 4: message_kernel<4><<<grid, kBlock, 0, st>>>(n, nd, bits, y, m); break;
        case 8: message_kernel<8><<<grid, kBlock, 0, st>>>(n, nd, bits, y, m); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ldpc
