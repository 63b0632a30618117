// Learned surrogate of the reweight factor: MLP kernels on the gfx950 matrix
// cores (bfloat16 operands, float32 accumulation), training by Adam, and
// surrogate reweighting with an exact audit used as a control variate.
//
// Network: x (24 momentum components / (sqrt(s)/2), (kappa-1)/0.2; padded
// to 64 columns) -> 4 x [256, SiLU] -> h; yhat = (kappa - 1) h approximates
// log(|M_kappa|^2 / |M_base|^2).  Rows are (event, point) samples.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mgrw_internal.h"

namespace mgrw {

namespace {

constexpr int H = 256;                 // hidden width
constexpr int K0 = 64;                 // padded input width
constexpr int NRAW = 25;               // momentum components and kappa
constexpr int NFEAT = NRAW + 2 * 14;   // plus 2 p_i.p_j / s and its logarithm for 14 pairs
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + int64_t(H) * K0;
constexpr int64_t OFF_W2 = OFF_B1 + H;
constexpr int64_t OFF_B2 = OFF_W2 + int64_t(H) * H;
constexpr int64_t OFF_W3 = OFF_B2 + H;
constexpr int64_t OFF_B3 = OFF_W3 + int64_t(H) * H;
constexpr int64_t OFF_W4 = OFF_B3 + H;
constexpr int64_t OFF_B4 = OFF_W4 + int64_t(H) * H;
constexpr int64_t OFF_W5 = OFF_B4 + H;
constexpr int64_t OFF_B5 = OFF_W5 + H;
constexpr int64_t NPAR = OFF_B5 + 1;
constexpr char kCheckpointMagic[9] = "MGRWSUR1";
static_assert(NPAR == MGRW_SURROGATE_N_PARAMS, "parameter layout");

constexpr int64_t W_OFF[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4};
constexpr int64_t B_OFF[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
constexpr int K_IN[4] = {K0, H, H, H};

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// float -> bfloat16 bits, round to nearest even (the hardware conversion)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
// two floats -> two bfloat16 in one 32-bit word (a in the low half)
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    typedef __attribute__((ext_vector_type(2))) float f32x2;
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// 1 / (1 + e^-z) with the hardware reciprocal (1 ulp): the activation is
// rounded to bfloat16 afterwards
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float dsilu(float z) {
    float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

// Counter-based uniform draws in (0, 1): SplitMix64 finaliser of
// (seed, stream, index); the same on the host and the device.
__host__ __device__ inline uint64_t smix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline double u01(uint64_t seed, uint64_t stream, uint64_t i) {
    uint64_t h = smix(seed + 0x9E3779B97F4A7C15ull * (stream + 1));
    h = smix(h + 0x9E3779B97F4A7C15ull * (i + 1));
    return (double(h >> 11) + 0.5) * 0x1.0p-53;
}

// ------------------------------------------------------------------ GEMM
//
// C[m][n] = sum_k A(m, k) B(k, n), bfloat16 operands, float accumulation,
// on v_mfma_f32_32x32x16_bf16.  A(m, k) = A[m*sam + k*sak], B(k, n) =
// B[k*sbk + n*sbn]; AKC (BKC): k is the contiguous index of A (B), else m (n)
// is.  Tile 64 x 64 x 32 per 256-thread workgroup, each wave a 32 x 32 block;
// grid (M/64, N/64, split-K slices).  M, N multiples of 64, K and the slice
// multiples of 32.
constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;

enum { EPI_F32 = 0, EPI_FWD = 1, EPI_BWD = 2 };

struct epi_args {
    float* c;             // EPI_F32: C[slice][M][N]
    const float* bias;    // EPI_FWD: bias[N]
    float* zout;          // EPI_FWD: pre-activation (may be null)
    uint16_t* aout;       // EPI_FWD: SiLU(z), bfloat16; EPI_BWD: dz, bfloat16
    const float* zin;     // EPI_BWD: pre-activation of the layer below
};

template <bool AKC>
__device__ __forceinline__ void load_tile(uint16_t (*S)[LDK], const uint16_t* __restrict__ G, int64_t s_mn,
                                          int64_t s_k, int mn0, int k0, int t) {
    if (AKC) {   // 64 rows x 32 k, k contiguous: 8 k per thread
        int r = t >> 2, c = (t & 3) * 8;
        uint4 v = *reinterpret_cast<const uint4*>(G + int64_t(mn0 + r) * s_mn + (k0 + c));
        *reinterpret_cast<uint4*>(&S[r][c]) = v;
    } else {     // 32 k x 64 rows, rows contiguous: 8 rows per thread, transposed into LDS
        int kk = t >> 3, r = (t & 7) * 8;
        uint4 v = *reinterpret_cast<const uint4*>(G + int64_t(k0 + kk) * s_k + (mn0 + r));
        const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
        for (int j = 0; j < 8; ++j) S[r + j][kk] = e[j];
    }
}

template <bool AKC, bool BKC, int EPI>
__global__ void __launch_bounds__(256)
gemm_bf16(const uint16_t* __restrict__ A, int64_t sam, int64_t sak, const uint16_t* __restrict__ B, int64_t sbk,
          int64_t sbn, int M, int N, int K, int kslice, epi_args ep) {
    __shared__ uint16_t As[BM][LDK];
    __shared__ uint16_t Bs[BN][LDK];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kb = blockIdx.z * kslice, ke = min(K, kb + kslice);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x16 acc = {};
    for (int k0 = kb; k0 < ke; k0 += BK) {
        load_tile<AKC>(As, A, sam, sak, m0, k0, t);
        load_tile<BKC>(Bs, B, sbn, sbk, n0, k0, t);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm + (lane & 31)][kk + (lane >> 5) * 8]);
            bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn + (lane & 31)][kk + (lane >> 5) * 8]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int col = n0 + wn + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const int64_t idx = int64_t(row) * N + col;
        if (EPI == EPI_F32) {
            ep.c[int64_t(blockIdx.z) * M * N + idx] = acc[r];
        } else if (EPI == EPI_FWD) {
            float z = acc[r] + ep.bias[col];
            if (ep.zout) ep.zout[idx] = z;
            ep.aout[idx] = f2bf(silu(z));
        } else {
            ep.aout[idx] = f2bf(acc[r] * dsilu(ep.zin[idx]));
        }
    }
}

// ------------------------------------------------------- elementwise kernels

// Feature rows r = e*P + k of events [e0, e0 + rows/P): bfloat16 x[r][64],
// kd[r] = kappa_k - 1.  Features: the 24 momentum components over sqrt(s)/2,
// (kappa - 1)/0.2, then for the 14 particle pairs (i < j) other than the two
// beams v_ij = 2 p_i.p_j / s and log(v_ij); absent particles give zeros.
// The points' kappa values travel by value with each launch.
struct kappa_set {
    double k[MGRW_MAX_POINTS];
};

__global__ void features_kernel(const double* __restrict__ mom, int n_ext, int64_t n, int64_t e0, int P,
                                kappa_set kappa, int64_t rows, uint16_t* __restrict__ x, float* __restrict__ kd) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int64_t e = e0 + r / P;
    const int k = int(r % P);
    const double rs = mom[0 * n + e] + mom[int64_t(4) * n + e];   // sqrt(s) = E1 + E2 in the CM frame
    const double inv = 2.0 / rs;
    uint16_t* xr = x + r * K0;
    for (int i = 0; i < 24; ++i) xr[i] = i < n_ext * 4 ? f2bf(float(mom[int64_t(i) * n + e] * inv)) : uint16_t(0);
    xr[24] = f2bf(float((kappa.k[k] - 1.0) / 0.2));
    int c = NRAW;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j) {
            if (i == 0 && j == 1) continue;
            float v = 0.0f, lv = 0.0f;
            if (j < n_ext) {
                const double* pi = mom + int64_t(i) * 4 * n + e;
                const double* pj = mom + int64_t(j) * 4 * n + e;
                const double d = pi[0] * pj[0] - pi[n] * pj[n] - pi[2 * n] * pj[2 * n] - pi[3 * n] * pj[3 * n];
                const double u = 2.0 * d / (rs * rs);
                v = float(u);
                lv = float(log(fmax(u, 1e-12)));
            }
            xr[c] = f2bf(v);
            xr[c + 14] = f2bf(lv);
            ++c;
        }
    for (int i = NFEAT; i < K0; ++i) xr[i] = 0;
    kd[r] = float(kappa.k[k] - 1.0);
}

// Gather training samples s = perm[b0 + r]: event s / P, point s % P, from
// features precomputed for all samples.
__global__ void gather_kernel(const int32_t* __restrict__ perm, int64_t b0, int rows,
                              const uint16_t* __restrict__ xall, const float* __restrict__ kdall,
                              const float* __restrict__ yall, uint16_t* __restrict__ x, float* __restrict__ kd,
                              float* __restrict__ y) {
    const int t = threadIdx.x;
    const int r = blockIdx.x;
    if (r >= rows) return;
    const int64_t s = perm[b0 + r];
    if (t < K0 / 8)
        reinterpret_cast<uint4*>(x + int64_t(r) * K0)[t] = reinterpret_cast<const uint4*>(xall + s * K0)[t];
    if (t == 0) {
        kd[r] = kdall[s];
        y[r] = yall[s];
    }
}

// Feature rows of given float features [m][NFEAT] (tests).
__global__ void features_from_f32(const float* __restrict__ xin, int64_t m, uint16_t* __restrict__ x) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= m) return;
    for (int i = 0; i < K0; ++i) x[r * K0 + i] = i < NFEAT ? f2bf(xin[r * NFEAT + i]) : uint16_t(0);
}

// Output layer, 64 rows per block (4 threads per row): h = a4 . w5 + b5,
// yhat = kd h.  Training: loss, dz4 = dh w5 silu'(z4) with dh = 2 (yhat - y)
// kd / m_total, and block partials of dw5, db5.  Inference: w_out.
template <bool TRAIN>
__global__ void __launch_bounds__(256)
head_kernel(const uint16_t* __restrict__ a4, const float* __restrict__ z4, const float* __restrict__ w5,
            const float* __restrict__ b5, const float* __restrict__ kd, const float* __restrict__ y, int64_t m,
            double inv_m_total, float* __restrict__ pred, uint16_t* __restrict__ dz4,
            float* __restrict__ dw5_part, double* __restrict__ loss_acc,
            // inference
            int P, int64_t n_events, int64_t e0, const double* __restrict__ w_in, double* __restrict__ w_out) {
    __shared__ float red[H + 1];
    const int t = threadIdx.x, q = t & 3;
    const int64_t row = int64_t(blockIdx.x) * 64 + (t >> 2);
    if (TRAIN) {
        for (int i = t; i <= H; i += 256) red[i] = 0.0f;
        __syncthreads();
    }
    const bool ok = row < m;
    float h = 0.0f;
    if (ok) {
        const uint16_t* ar = a4 + row * H + q * 64;
        for (int j = 0; j < 64; ++j) h += bf2f(ar[j]) * w5[q * 64 + j];
    }
    h += __shfl_xor(h, 1);
    h += __shfl_xor(h, 2);
    h += b5[0];
    const float kr = ok ? kd[row] : 0.0f;
    const float yh = kr * h;
    if (!TRAIN) {
        if (ok && q == 0) {
            const int64_t e = e0 + row / P;
            const int k = int(row % P);
            const double w = w_in ? w_in[e] : 1.0;
            w_out[int64_t(k) * n_events + e] = w * exp(double(yh));
            if (pred) pred[row] = yh;
        }
        return;
    }
    float dh = 0.0f;
    if (ok) {
        const float diff = yh - y[row];
        dh = float(2.0 * double(diff) * inv_m_total) * kr;
        if (q == 0) {
            pred[row] = yh;
            atomicAdd(loss_acc, double(diff) * double(diff) * inv_m_total);
            atomicAdd(&red[H], dh);
        }
        const uint16_t* ar = a4 + row * H + q * 64;
        const float* zr = z4 + row * H + q * 64;
        uint16_t* dr = dz4 + row * H + q * 64;
        for (int j = 0; j < 64; ++j) {
            dr[j] = f2bf(dh * w5[q * 64 + j] * dsilu(zr[j]));
            atomicAdd(&red[q * 64 + j], dh * bf2f(ar[j]));
        }
    }
    __syncthreads();
    for (int i = t; i <= H; i += 256) dw5_part[int64_t(blockIdx.x) * (H + 1) + i] = red[i];
}

// out[i] = sum over s of part[s][i]  (split-K and block partials)
__global__ void reduce_parts(const float* __restrict__ part, int nparts, int64_t len, float* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += part[int64_t(p) * len + i];
    out[i] = s;
}

// out[i] = sum over s of part[s][i] for many partials of a short row (bias
// and output-layer gradients): one workgroup per column i, its 256 threads
// taking partials s = t, t + 256, ..., then a fixed-order tree; deterministic.
__global__ void __launch_bounds__(256)
reduce_cols(const float* __restrict__ part, int nparts, int64_t len, float* __restrict__ out) {
    const int t = threadIdx.x;
    const int64_t i = blockIdx.x;
    float s = 0.0f;
    for (int p = t; p < nparts; p += 256) s += part[int64_t(p) * len + i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ float w[4];
    if ((t & 63) == 0) w[t >> 6] = s;
    __syncthreads();
    if (t == 0) out[i] = (w[0] + w[1]) + (w[2] + w[3]);
}

// Row chunks of the bias-gradient column sums: enough workgroups to spread
// over the 256 CUs, few enough for one pass of the final reduction.
constexpr int kBiasChunks = 256;

// Partial column sums of a bfloat16 [m][H] matrix (bias gradients): block b
// sums rows [b*rows_per, (b+1)*rows_per) of every column; deterministic.
__global__ void colsum_bf16(const uint16_t* __restrict__ g, int64_t m, int64_t rows_per, float* __restrict__ part) {
    const int c = threadIdx.x;
    const int64_t r0 = int64_t(blockIdx.x) * rows_per, r1 = min(m, r0 + rows_per);
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += bf2f(g[r * H + c]);
    part[int64_t(blockIdx.x) * H + c] = s;
}

// Adam on the float32 master parameters; refresh the bfloat16 copy.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, uint16_t* __restrict__ pbf, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float v = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    p[i] = v;
    pbf[i] = f2bf(v);
}

__global__ void to_bf16(const float* __restrict__ p, int64_t n, uint16_t* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(p[i]);
}

// y = log(w) of the exact reweight output [P][n] into sample order s = e*P + k.
__global__ void labels_kernel(const double* __restrict__ w, int P, int64_t n, float* __restrict__ y) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n * P) return;
    const int64_t e = s / P;
    const int k = int(s % P);
    y[s] = float(log(w[int64_t(k) * n + e]));
}

__global__ void gather_events(const double* __restrict__ mom, int n_ext, int64_t n, const int64_t* __restrict__ idx,
                              int64_t na, const double* __restrict__ w_in, double* __restrict__ mom_a,
                              double* __restrict__ w_a) {
    const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= na) return;
    const int64_t e = idx[a];
    for (int c = 0; c < n_ext * 4; ++c) mom_a[int64_t(c) * na + a] = mom[int64_t(c) * n + e];
    w_a[a] = w_in ? w_in[e] : 1.0;
}

// Per point k: partial sums over events of the surrogate weights.
__global__ void sum_rows(const double* __restrict__ w, int P, int64_t n, double* __restrict__ part) {
    __shared__ double red[256];
    const int k = blockIdx.y;
    double s = 0.0;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
        s += w[int64_t(k) * n + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[int64_t(k) * gridDim.x + blockIdx.x] = red[0];
}

// Audit: per point, sums over audited events of (exact - surrogate), and of
// the relative error |su/ex - 1| and its square with the number of events
// entering them (those with a finite non-zero exact weight and a finite
// ratio: a zero input weight makes both weights zero, |M|^2 = 0 at the base
// makes the exact one NaN); then the exact weights replace the surrogate
// ones.  One block per point (audits are small).
__global__ void audit_kernel(const int64_t* __restrict__ idx, int64_t na, const double* __restrict__ w_exact,
                             int64_t n, double* __restrict__ w_out, double* __restrict__ stats) {
    __shared__ double red[4][256];
    const int k = blockIdx.x;
    double d = 0.0, e1 = 0.0, e2 = 0.0, m = 0.0;
    for (int64_t a = threadIdx.x; a < na; a += 256) {
        const double ex = w_exact[int64_t(k) * na + a];
        const double su = w_out[int64_t(k) * n + idx[a]];
        d += ex - su;
        const double r = fabs(su / ex - 1.0);
        if (ex != 0.0 && isfinite(r)) {
            e1 += r;
            e2 += r * r;
            m += 1.0;
        }
    }
    red[0][threadIdx.x] = d;
    red[1][threadIdx.x] = e1;
    red[2][threadIdx.x] = e2;
    red[3][threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int j = 0; j < 4; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int j = 0; j < 4; ++j) stats[k * 4 + j] = red[j][0];
    __syncthreads();
    for (int64_t a = threadIdx.x; a < na; a += 256) w_out[int64_t(k) * n + idx[a]] = w_exact[int64_t(k) * na + a];
}

// ------------------------------------------------- fused inference
//
// All four hidden layers and the output unit for 128 feature rows per
// workgroup.  The rows' activations stay in one LDS buffer (128 x 256
// bfloat16, 67.6 KB, so two workgroups share a CU and one's epilogue overlaps
// the other's matrix work), updated in place: each wave computes 64 units x
// 128 rows of a layer into registers on v_mfma_f32_32x32x16_bf16, the
// workgroup synchronises, and the epilogue (bias, SiLU, rounding to bfloat16)
// overwrites the layer's input.  The product is D = W A^T: the weights (rows
// of the L2-resident bfloat16 copy, each read once per workgroup) are the
// first operand, the activations the second, so a lane's four consecutive
// accumulator rows are four consecutive units of one feature row, stored as
// one 8-byte word.  Rows are event-major (r = e P + k): layer 1 reads the
// event's features (computed once per event) and the point's kappa.  Same
// arithmetic as the layer-by-layer training kernels.  rows < 2^31.
constexpr int FR = 128;         // rows per workgroup
constexpr int LDA = H + 8;      // LDS row stride (bfloat16)

__global__ void __launch_bounds__(256, 2)
mlp_infer_kernel(const uint16_t* __restrict__ xev, int P, kappa_set kappa, int rows, int64_t e0,
                 int64_t n_events, const uint16_t* __restrict__ wbf, const float* __restrict__ par,
                 const double* __restrict__ w_in, double* __restrict__ w_out) {
    __shared__ __align__(16) uint16_t act[FR][LDA];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, lr = lane & 31, lh = lane >> 5;
    const int r0 = int(blockIdx.x) * FR;
    {
        // layer-1 input: 2 threads per row, 32 columns each
        const int mrow = t >> 1, q = t & 1, r = r0 + mrow;
        const bool live = r < rows;
        const uint4* src = reinterpret_cast<const uint4*>(xev + int64_t((live ? r : 0) / P) * K0 + q * 32);
        uint4* dst = reinterpret_cast<uint4*>(&act[mrow][q * 32]);
#pragma unroll
        for (int i = 0; i < 4; ++i) dst[i] = live ? src[i] : make_uint4(0u, 0u, 0u, 0u);
        if (q == 0 && r < rows) act[mrow][NRAW - 1] = f2bf(float((kappa.k[r % P] - 1.0) / 0.2));
    }
    __syncthreads();
#pragma unroll 1
    for (int l = 0; l < 4; ++l) {
        const int K = K_IN[l];
        const uint16_t* W = wbf + W_OFF[l];   // [H][K]
        const float* bias = par + B_OFF[l];
        f32x16 acc[2][4];   // [unit tile][row tile]
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) acc[ut][rt] = f32x16{};
#pragma unroll 2
        for (int ks = 0; ks < K / 16; ++ks) {
            bf16x8 w[2], x[4];
#pragma unroll
            for (int ut = 0; ut < 2; ++ut)
                w[ut] = *reinterpret_cast<const bf16x8*>(W + ((wave * 2 + ut) * 32 + lr) * K + ks * 16 + lh * 8);
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) x[rt] = *reinterpret_cast<const bf16x8*>(&act[rt * 32 + lr][ks * 16 + lh * 8]);
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int ut = 0; ut < 2; ++ut)
                    acc[ut][rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[ut], x[rt], acc[ut][rt], 0, 0, 0);
        }
        __syncthreads();   // every wave has read the layer's input
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int n = (wave * 2 + ut) * 32 + g * 8 + lh * 4;   // units n .. n+3
                const float4 bn = *reinterpret_cast<const float4*>(bias + n);
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const f32x16& c = acc[ut][rt];
                    const uint32_t lo = pack_bf16(silu(c[4 * g] + bn.x), silu(c[4 * g + 1] + bn.y));
                    const uint32_t hi = pack_bf16(silu(c[4 * g + 2] + bn.z), silu(c[4 * g + 3] + bn.w));
                    *reinterpret_cast<uint2*>(&act[rt * 32 + lr][n]) = make_uint2(lo, hi);
                }
            }
        __syncthreads();
    }
    // output unit on the last hidden layer; two threads per row
    const int mrow = t >> 1, q = t & 1;
    float h = 0.0f;
    const float4* w5 = reinterpret_cast<const float4*>(par + OFF_W5 + q * 128);
    const uint4* ar = reinterpret_cast<const uint4*>(&act[mrow][q * 128]);
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const uint4 a8 = ar[j];
        const float4 wa = w5[2 * j], wb = w5[2 * j + 1];
        h += __uint_as_float(a8.x << 16) * wa.x + __uint_as_float(a8.x & 0xffff0000u) * wa.y;
        h += __uint_as_float(a8.y << 16) * wa.z + __uint_as_float(a8.y & 0xffff0000u) * wa.w;
        h += __uint_as_float(a8.z << 16) * wb.x + __uint_as_float(a8.z & 0xffff0000u) * wb.y;
        h += __uint_as_float(a8.w << 16) * wb.z + __uint_as_float(a8.w & 0xffff0000u) * wb.w;
    }
    h += __shfl_xor(h, 1);
    const int r = r0 + mrow;
    if (q == 0 && r < rows) {
        const int k = r % P;
        const int64_t e = e0 + r / P;
        const float yh = float(kappa.k[k] - 1.0) * (h + par[OFF_B5]);
        const double w = w_in ? w_in[e] : 1.0;
        w_out[int64_t(k) * n_events + e] = w * exp(double(yh));
    }
}

// Audit selection u01(seed, 2, e) < f, compacted in event order: per-block
// counts, one-workgroup exclusive scan, then each block writes its events.
__global__ void __launch_bounds__(256)
audit_count_kernel(uint64_t seed, double f, int64_t n, unsigned* __restrict__ counts) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool sel = e < n && u01(seed, 2, uint64_t(e)) < f;
    __shared__ unsigned c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    if (sel) atomicAdd(&c, 1u);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

__global__ void __launch_bounds__(256)
audit_scan_kernel(const unsigned* __restrict__ counts, int64_t nb, int64_t* __restrict__ offsets) {
    __shared__ int64_t tot[256];
    const int t = threadIdx.x;
    const int64_t per = (nb + 255) / 256, b0 = t * per, b1 = b0 + per < nb ? b0 + per : nb;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += counts[b];
    tot[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int i = 0; i < 256; ++i) {
            const int64_t v = tot[i];
            tot[i] = run;
            run += v;
        }
        offsets[nb] = run;   // total
    }
    __syncthreads();
    int64_t run = tot[t];
    for (int64_t b = b0; b < b1; ++b) {
        offsets[b] = run;
        run += counts[b];
    }
}

__global__ void __launch_bounds__(256)
audit_fill_kernel(uint64_t seed, double f, int64_t n, const int64_t* __restrict__ offsets, int64_t na,
                  int64_t* __restrict__ idx) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool sel = e < n && u01(seed, 2, uint64_t(e)) < f;
    __shared__ unsigned flags[256];
    flags[threadIdx.x] = sel ? 1u : 0u;
    __syncthreads();
    if (sel) {
        unsigned pos = 0;
        for (unsigned i = 0; i < threadIdx.x; ++i) pos += flags[i];
        const int64_t at = offsets[blockIdx.x] + pos;
        if (at < na) idx[at] = e;   // na: the same count, made on the host
    }
}

// --------------------------------------------------------------- host side

template <typename T>
struct dbuf {   // device buffer owned by the library
    T* p = nullptr;
    size_t n = 0;
    hipError_t alloc(size_t count) {
        if (count <= n) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e == hipSuccess) n = count;
        return e;
    }
    ~dbuf() {
        if (p) (void)hipFree(p);
    }
};

template <typename T>
struct sbuf {   // scratch of one call, allocated and freed in the order of its stream
    T* p = nullptr;
    hipStream_t s;
    explicit sbuf(hipStream_t st) : s(st) {}
    sbuf(const sbuf&) = delete;
    sbuf& operator=(const sbuf&) = delete;
    hipError_t alloc(size_t count) {
        return hipMallocAsync(reinterpret_cast<void**>(&p), std::max<size_t>(count, 1) * sizeof(T), s);
    }
    ~sbuf() {
        if (p) (void)hipFreeAsync(p, s);
    }
};

}  // namespace

struct surrogate {
    dbuf<float> par, grad, m1, m2;
    dbuf<uint16_t> pbf;
    // activations of one batch
    dbuf<uint16_t> x0, act[4], dz[2];
    dbuf<float> z[4], kd, y, pred, part;
    dbuf<double> lossd;
    int64_t rows_cap = 0;
    int step = 0;
};

void surrogate_destroy(surrogate* s) { delete s; }

namespace {

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return set_error(MGRW_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

hipError_t ensure_rows(surrogate* s, int64_t rows) {
    if (rows <= s->rows_cap) return hipSuccess;
    hipError_t e;
    if ((e = s->x0.alloc(size_t(rows) * K0)) != hipSuccess) return e;
    for (int l = 0; l < 4; ++l) {
        if ((e = s->act[l].alloc(size_t(rows) * H)) != hipSuccess) return e;
        if ((e = s->z[l].alloc(size_t(rows) * H)) != hipSuccess) return e;
    }
    for (int l = 0; l < 2; ++l)
        if ((e = s->dz[l].alloc(size_t(rows) * H)) != hipSuccess) return e;
    if ((e = s->kd.alloc(rows)) != hipSuccess) return e;
    if ((e = s->y.alloc(rows)) != hipSuccess) return e;
    if ((e = s->pred.alloc(rows)) != hipSuccess) return e;
    // split-K partials (<= 16 slices of H x H), output-layer block partials,
    // and bias-gradient partials (<= kBiasChunks row chunks)
    if ((e = s->part.alloc(std::max<size_t>(size_t(16) * H * H, size_t(rows / 64 + 1) * (H + 1)) +
                           size_t(kBiasChunks) * H)) != hipSuccess)
        return e;
    s->rows_cap = rows;
    return hipSuccess;
}

mgrw_status new_surrogate(mgrw_process* p) {
    if (!p->sur) {
        p->sur = new (std::nothrow) surrogate;
        if (!p->sur) return set_error(MGRW_ERR_ALLOC, "out of host memory");
    }
    surrogate* s = p->sur;
    HIPCHK(s->par.alloc(NPAR));
    HIPCHK(s->grad.alloc(NPAR));
    HIPCHK(s->m1.alloc(NPAR));
    HIPCHK(s->m2.alloc(NPAR));
    HIPCHK(s->pbf.alloc(NPAR));
    HIPCHK(s->lossd.alloc(1));
    return MGRW_OK;
}

void init_params(std::vector<float>& w, uint64_t seed) {
    w.assign(NPAR, 0.0f);
    int64_t i = 0;
    auto fill = [&](int64_t off, int rows, int cols, int used_cols, double scale) {
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c)
                w[off + int64_t(r) * cols + c] =
                    c < used_cols ? float((2.0 * u01(seed, 3, uint64_t(i++)) - 1.0) * scale) : 0.0f;
    };
    fill(OFF_W1, H, K0, NFEAT, std::sqrt(6.0 / NFEAT));
    fill(OFF_W2, H, H, H, std::sqrt(6.0 / H));
    fill(OFF_W3, H, H, H, std::sqrt(6.0 / H));
    fill(OFF_W4, H, H, H, std::sqrt(6.0 / H));
    fill(OFF_W5, 1, H, H, 0.1 / std::sqrt(double(H)));
}

template <bool AKC, bool BKC, int EPI>
void gemm(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk, int64_t sbn, int M, int N,
          int K, int splits, const epi_args& ep, hipStream_t s) {
    dim3 grid(M / BM, N / BN, splits);
    hipLaunchKernelGGL((gemm_bf16<AKC, BKC, EPI>), grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, M, N, K,
                       K / splits, ep);
}

// Forward through the hidden layers for `rows` feature rows in s->x0.
void forward(surrogate* s, int64_t rows, bool keep_z, hipStream_t st) {
    const uint16_t* in = s->x0.p;
    for (int l = 0; l < 4; ++l) {
        epi_args ep{};
        ep.bias = s->par.p + B_OFF[l];
        ep.zout = keep_z ? s->z[l].p : nullptr;
        ep.aout = s->act[l].p;
        // Z[m][n] = sum_k X[m][k] W[n][k]: A = X (k contiguous), B(k, n) = W[n*K + k] (k contiguous)
        gemm<true, true, EPI_FWD>(in, K_IN[l], 1, s->pbf.p + W_OFF[l], 1, K_IN[l], int(rows), H, K_IN[l], 1, ep,
                                  st);
        in = s->act[l].p;
    }
}

// Backward for one batch whose dz4 is in s->dz[0]; gradients into s->grad.
mgrw_status backward(surrogate* s, int64_t rows, hipStream_t st) {
    int cur = 0;
    int splits = 16;   // split-K slices: each a multiple of 32 rows
    while (splits > 1 && rows % (int64_t(32) * splits) != 0) --splits;
    const int nchunk = int(std::min<int64_t>(kBiasChunks, rows));
    const int64_t rows_per = (rows + nchunk - 1) / nchunk;
    float* bias_part = s->part.p + size_t(16) * H * H;
    for (int l = 3; l >= 0; --l) {
        const uint16_t* dzl = s->dz[cur].p;
        const uint16_t* below = l > 0 ? s->act[l - 1].p : s->x0.p;
        const int kin = K_IN[l];
        // dW[n][k] = sum_m dz[m][n] a[m][k]: A(n, m) = dz[m*H + n] (n contiguous),
        // B(m, k) = a[m*kin + k] (k = output column contiguous)
        epi_args ep{};
        ep.c = s->part.p;
        gemm<false, false, EPI_F32>(dzl, 1, H, below, kin, 1, H, kin, int(rows), splits, ep, st);
        hipLaunchKernelGGL(reduce_parts, dim3(unsigned((H * kin + 255) / 256)), dim3(256), 0, st, s->part.p, splits,
                           int64_t(H) * kin, s->grad.p + W_OFF[l]);
        hipLaunchKernelGGL(colsum_bf16, dim3(unsigned(nchunk)), dim3(H), 0, st, dzl, rows, rows_per, bias_part);
        hipLaunchKernelGGL(reduce_cols, dim3(H), dim3(256), 0, st, bias_part, nchunk, int64_t(H),
                           s->grad.p + B_OFF[l]);
        if (l > 0) {
            // da[m][k] = sum_n dz[m][n] W[n][k]: A = dz (n contiguous as k), B(n, k) = W[n*H + k]
            // (k = output column contiguous); fused with silu'(z) of layer l-1
            epi_args eb{};
            eb.aout = s->dz[1 - cur].p;
            eb.zin = s->z[l - 1].p;
            gemm<true, false, EPI_BWD>(dzl, H, 1, s->pbf.p + W_OFF[l], H, 1, int(rows), H, H, 1, eb, st);
            cur = 1 - cur;
        }
    }
    HIPCHK(hipGetLastError());
    return MGRW_OK;
}

// Loss, output layer and its backward for one batch.
mgrw_status head_train(surrogate* s, int64_t rows, double inv_m, hipStream_t st) {
    const unsigned blocks = unsigned((rows + 63) / 64);
    hipLaunchKernelGGL((head_kernel<true>), dim3(blocks), dim3(256), 0, st, s->act[3].p, s->z[3].p,
                       s->par.p + OFF_W5, s->par.p + OFF_B5, s->kd.p, s->y.p, rows, inv_m, s->pred.p, s->dz[0].p,
                       s->part.p, s->lossd.p, 0, int64_t(0), int64_t(0), nullptr, nullptr);
    // dw5 and db5 from the block partials (w5 and b5 are contiguous)
    hipLaunchKernelGGL(reduce_cols, dim3(H + 1), dim3(256), 0, st, s->part.p, int(blocks), int64_t(H + 1),
                       s->grad.p + OFF_W5);
    HIPCHK(hipGetLastError());
    return MGRW_OK;
}

void adam(surrogate* s, float lr, hipStream_t st) {
    s->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, float(s->step)), c2 = 1.0f - std::pow(b2, float(s->step));
    hipLaunchKernelGGL(adam_kernel, dim3(unsigned((NPAR + 255) / 256)), dim3(256), 0, st, s->par.p, s->grad.p,
                       s->m1.p, s->m2.p, s->pbf.p, NPAR, lr, b1, b2, 1e-8f, c1, c2);
}

mgrw_status check_qcd_kappa_only(const mgrw_process* p) {
    if (p->proc == MGRW_EE_MUMU || p->proc == MGRW_EE_5A)
        return set_error(MGRW_ERR_UNSUPPORTED, "surrogate: QCD processes only");
    // the network's output (kappa - 1) h and its kappa feature vanish at
    // kappa = 1, where the target log(|M_k|^2 / |M_base|^2) must vanish too
    if (p->base.kappa_ttg != 1.0)
        return set_error(MGRW_ERR_UNSUPPORTED, "surrogate: the base point must have kappa_ttg = 1");
    if (p->n_points == 0) return set_error(MGRW_ERR_STATE, "no parameter points set");
    for (int k = 0; k < p->n_points; ++k) {
        const mgrw_params& q = p->points[k];
        if (q.alphas != p->base.alphas || q.mt != p->base.mt)
            return set_error(MGRW_ERR_UNSUPPORTED, "surrogate: points may only change kappa_ttg");
    }
    return MGRW_OK;
}

kappa_set kappas_of(const mgrw_process* p) {
    kappa_set k{};
    for (int i = 0; i < p->n_points; ++i) k.k[i] = p->points[i].kappa_ttg;
    return k;
}

// Number of events with u(seed, 2, e) < f: the audit set's size, the same
// draw the device makes (computed here so that the call need not wait for
// the device before sizing the audit).
int64_t audit_size(uint64_t seed, double f, int64_t n) {
    int64_t c = 0;
    for (int64_t e = 0; e < n; ++e) c += u01(seed, 2, uint64_t(e)) < f;
    return c;
}

// Fit a freshly initialised network (seeded) to ns samples: bfloat16
// feature rows xall [ns][64], kd = kappa - 1, targets y; Adam on shuffled
// batches, per-epoch mean loss into loss_out (host, may be NULL).
mgrw_status train_core(mgrw_process* p, const uint16_t* xall, const float* kdall, const float* yall, int64_t ns,
                       const mgrw_train_config* cfg, double* loss_out, hipStream_t st) {
    std::vector<float> w0;
    init_params(w0, cfg->seed);
    mgrw_status r = mgrw_surrogate_set(p, w0.data());
    if (r != MGRW_OK) return r;
    surrogate* s = p->sur;
    const int64_t B = cfg->batch;
    HIPCHK(ensure_rows(s, B));
    const int64_t nb = ns / B;
    if (nb < 1) return set_error(MGRW_ERR_ARG, "fewer samples than one batch");
    std::vector<int32_t> perm(ns);
    dbuf<int32_t> dperm;
    HIPCHK(dperm.alloc(size_t(ns)));
    float lr = float(cfg->lr);
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        for (int64_t i = 0; i < ns; ++i) perm[i] = int32_t(i);
        for (int64_t i = ns - 1; i > 0; --i) {   // Fisher-Yates with a counter-based generator
            int64_t j = int64_t(u01(cfg->seed + 7919 * uint64_t(ep + 1), 3, uint64_t(i)) * double(i + 1));
            if (j > i) j = i;
            std::swap(perm[i], perm[j]);
        }
        HIPCHK(hipMemcpyAsync(dperm.p, perm.data(), size_t(ns) * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemsetAsync(s->lossd.p, 0, sizeof(double), st));
        for (int64_t b = 0; b < nb; ++b) {
            hipLaunchKernelGGL(gather_kernel, dim3(unsigned(B)), dim3(64), 0, st, dperm.p, b * B, int(B), xall,
                               kdall, yall, s->x0.p, s->kd.p, s->y.p);
            forward(s, B, true, st);
            r = head_train(s, B, 1.0 / double(B), st);
            if (r != MGRW_OK) return r;
            r = backward(s, B, st);
            if (r != MGRW_OK) return r;
            adam(s, lr, st);
        }
        double lsum = 0.0;
        HIPCHK(hipMemcpyAsync(&lsum, s->lossd.p, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (loss_out) loss_out[ep] = lsum / double(nb);
        lr *= float(cfg->lr_decay);
    }
    HIPCHK(hipGetLastError());
    return MGRW_OK;
}

}  // namespace
}  // namespace mgrw

using namespace mgrw;

extern "C" {

mgrw_status mgrw_surrogate_set(mgrw_process* p, const float* params) {
    if (!p || !params) return set_error(MGRW_ERR_ARG, "null argument");
    mgrw_status st = new_surrogate(p);
    if (st != MGRW_OK) return st;
    surrogate* s = p->sur;
    HIPCHK(hipMemcpy(s->par.p, params, NPAR * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(s->m1.p, 0, NPAR * sizeof(float)));
    HIPCHK(hipMemset(s->m2.p, 0, NPAR * sizeof(float)));
    s->step = 0;
    hipLaunchKernelGGL(to_bf16, dim3(unsigned((NPAR + 255) / 256)), dim3(256), 0, 0, s->par.p, NPAR, s->pbf.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    return MGRW_OK;
}

mgrw_status mgrw_surrogate_get(const mgrw_process* p, float* params) {
    if (!p || !params) return set_error(MGRW_ERR_ARG, "null argument");
    if (!p->sur || !p->sur->par.p) return set_error(MGRW_ERR_STATE, "no surrogate");
    HIPCHK(hipMemcpy(params, p->sur->par.p, NPAR * sizeof(float), hipMemcpyDeviceToHost));
    return MGRW_OK;
}

mgrw_status mgrw_surrogate_save(const mgrw_process* p, const char* path) {
    if (!p || !path) return set_error(MGRW_ERR_ARG, "null argument");
    if (!p->sur || !p->sur->par.p) return set_error(MGRW_ERR_STATE, "no surrogate");
    std::vector<float> w(static_cast<size_t>(NPAR));
    mgrw_status st = mgrw_surrogate_get(p, w.data());
    if (st != MGRW_OK) return st;
    const std::string tmp = std::string(path) + ".part";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return set_error(MGRW_ERR_ARG, std::string("cannot write ") + tmp);
    const uint32_t head[2] = {uint32_t(NPAR), 0u};
    bool ok = std::fwrite(kCheckpointMagic, 1, 8, f) == 8 && std::fwrite(head, sizeof head, 1, f) == 1 &&
              std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
    if (std::fclose(f) != 0) ok = false;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return set_error(MGRW_ERR_ARG, std::string("writing ") + path + " failed");
    }
    return MGRW_OK;
}

mgrw_status mgrw_surrogate_load(mgrw_process* p, const char* path) {
    if (!p || !path) return set_error(MGRW_ERR_ARG, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(MGRW_ERR_ARG, std::string("cannot open ") + path);
    char magic[8];
    uint32_t head[2];
    std::vector<float> w(static_cast<size_t>(NPAR));
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kCheckpointMagic, 8) == 0 &&
              std::fread(head, sizeof head, 1, f) == 1 && head[0] == uint32_t(NPAR) &&
              std::fread(w.data(), sizeof(float), w.size(), f) == w.size();
    const bool at_end = ok && std::fgetc(f) == EOF;
    std::fclose(f);
    if (!ok || !at_end)
        return set_error(MGRW_ERR_ARG, std::string(path) + ": not a surrogate checkpoint of " +
                                           std::to_string(NPAR) + " parameters");
    return mgrw_surrogate_set(p, w.data());
}

mgrw_status mgrw_surrogate_fwd_bwd(mgrw_process* p, const float* x, const float* kd, const float* y, int64_t m,
                                   float* pred, float* grad, double* loss, void* stream) {
    if (!p || !x || !kd || !y || !pred || !grad || !loss) return set_error(MGRW_ERR_ARG, "null argument");
    if (m <= 0 || m % 64 != 0 || m > (int64_t(1) << 24)) return set_error(MGRW_ERR_ARG, "m must be a positive multiple of 64");
    if (!p->sur || !p->sur->par.p) return set_error(MGRW_ERR_STATE, "no surrogate");
    if (check_device_ptr(x, "x", false) != MGRW_OK || check_device_ptr(kd, "kd", false) != MGRW_OK ||
        check_device_ptr(y, "y", false) != MGRW_OK || check_device_ptr(pred, "pred", false) != MGRW_OK)
        return MGRW_ERR_ARG;
    surrogate* s = p->sur;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIPCHK(ensure_rows(s, m));
    hipLaunchKernelGGL(features_from_f32, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, x, m, s->x0.p);
    HIPCHK(hipMemcpyAsync(s->kd.p, kd, m * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(s->y.p, y, m * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(s->lossd.p, 0, sizeof(double), st));
    HIPCHK(hipMemsetAsync(s->grad.p, 0, NPAR * sizeof(float), st));
    forward(s, m, true, st);
    mgrw_status r = head_train(s, m, 1.0 / double(m), st);
    if (r != MGRW_OK) return r;
    r = backward(s, m, st);
    if (r != MGRW_OK) return r;
    HIPCHK(hipMemcpyAsync(pred, s->pred.p, m * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(grad, s->grad.p, NPAR * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(loss, s->lossd.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MGRW_OK;
}

mgrw_status mgrw_surrogate_train(mgrw_process* p, const double* mom, int64_t n_events, const mgrw_train_config* cfg,
                                 double* loss_out, void* stream) {
    if (!p || !cfg) return set_error(MGRW_ERR_ARG, "null argument");
    mgrw_status st0 = check_qcd_kappa_only(p);
    if (st0 != MGRW_OK) return st0;
    if (n_events <= 0 || !mom) return set_error(MGRW_ERR_ARG, "need events");
    if (cfg->epochs < 1 || cfg->batch < 64 || cfg->batch % 64 != 0 || !(cfg->lr > 0))
        return set_error(MGRW_ERR_ARG, "bad training configuration");
    const int P = p->n_points;
    const int64_t ns = n_events * P;
    if (ns >= (int64_t(1) << 31)) return set_error(MGRW_ERR_ARG, "too many samples");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int n_ext = 0;
    mgrw_process_info(p, &n_ext, nullptr, nullptr, nullptr);

    if (check_device_ptr(mom, "mom", false) != MGRW_OK) return MGRW_ERR_ARG;

    // labels from the exact kernels
    dbuf<double> wex;
    HIPCHK(wex.alloc(size_t(ns)));
    mgrw_status r = mgrw_reweight(p, mom, nullptr, n_events, wex.p, nullptr, stream);
    if (r != MGRW_OK) return r;
    dbuf<float> yall, kdall;
    dbuf<uint16_t> xall;
    HIPCHK(yall.alloc(size_t(ns)));
    HIPCHK(kdall.alloc(size_t(ns)));
    HIPCHK(xall.alloc(size_t(ns) * K0));
    hipLaunchKernelGGL(labels_kernel, dim3(unsigned((ns + 255) / 256)), dim3(256), 0, st, wex.p, P, n_events, yall.p);
    hipLaunchKernelGGL(features_kernel, dim3(unsigned((ns + 255) / 256)), dim3(256), 0, st, mom, n_ext, n_events,
                       int64_t(0), P, kappas_of(p), ns, xall.p, kdall.p);
    HIPCHK(hipGetLastError());

    return train_core(p, xall.p, kdall.p, yall.p, ns, cfg, loss_out, st);
}

mgrw_status mgrw_surrogate_train_samples(mgrw_process* p, const float* x, const float* kd, const float* y,
                                         int64_t m, const mgrw_train_config* cfg, double* loss_out, void* stream) {
    if (!p || !cfg || !x || !kd || !y) return set_error(MGRW_ERR_ARG, "null argument");
    if (m <= 0 || m >= (int64_t(1) << 31)) return set_error(MGRW_ERR_ARG, "m must be in [1, 2^31)");
    if (cfg->epochs < 1 || cfg->batch < 64 || cfg->batch % 64 != 0 || !(cfg->lr > 0))
        return set_error(MGRW_ERR_ARG, "bad training configuration");
    if (m < cfg->batch) return set_error(MGRW_ERR_ARG, "fewer samples than one batch");
    if (check_device_ptr(x, "x", false) != MGRW_OK || check_device_ptr(kd, "kd", false) != MGRW_OK ||
        check_device_ptr(y, "y", false) != MGRW_OK)
        return MGRW_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    dbuf<uint16_t> xall;
    dbuf<float> kdall, yall;
    HIPCHK(xall.alloc(size_t(m) * K0));
    HIPCHK(kdall.alloc(size_t(m)));
    HIPCHK(yall.alloc(size_t(m)));
    hipLaunchKernelGGL(features_from_f32, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, x, m, xall.p);
    HIPCHK(hipMemcpyAsync(kdall.p, kd, size_t(m) * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(yall.p, y, size_t(m) * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipGetLastError());
    return train_core(p, xall.p, kdall.p, yall.p, m, cfg, loss_out, st);
}

mgrw_status mgrw_reweight_surrogate(mgrw_process* p, const double* mom, const double* w_in, int64_t n_events,
                                    double audit_fraction, uint64_t seed, double max_audit_error, double* w_out,
                                    double* audit_stats, int* fell_back, void* stream) {
    if (!p) return set_error(MGRW_ERR_ARG, "process is NULL");
    mgrw_status r = check_qcd_kappa_only(p);
    if (r != MGRW_OK) return r;
    if (!p->sur || !p->sur->par.p) return set_error(MGRW_ERR_STATE, "no surrogate trained or loaded");
    if (!(audit_fraction > 0.0 && audit_fraction <= 1.0)) return set_error(MGRW_ERR_ARG, "audit_fraction not in (0, 1]");
    if (n_events < 0) return set_error(MGRW_ERR_ARG, "n_events < 0");
    if (fell_back) *fell_back = 0;
    if (n_events == 0) return MGRW_OK;
    if ((r = check_device_ptr(mom, "mom", false)) != MGRW_OK) return r;
    if ((r = check_device_ptr(w_out, "w_out", false)) != MGRW_OK) return r;
    if ((r = check_device_ptr(w_in, "w_in", true)) != MGRW_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    surrogate* s = p->sur;
    const int P = p->n_points;
    const kappa_set kap = kappas_of(p);
    int n_ext = 0;
    mgrw_process_info(p, &n_ext, nullptr, nullptr, nullptr);
    // Every buffer below is allocated and freed in stream order; the only
    // wait is for the audit statistics at the end.

    // 1. surrogate weights for every (event, point), in chunks of events: the
    // event features once per event, then the fused network over its P rows
    // (only the per-event features need a buffer: the activations stay in LDS)
    const int64_t chunk_ev = std::min<int64_t>(n_events, std::max<int64_t>(1, (int64_t(1) << 20) / P));
    sbuf<uint16_t> xev(st);
    sbuf<float> kdev(st);
    HIPCHK(xev.alloc(size_t(chunk_ev) * K0));
    HIPCHK(kdev.alloc(size_t(chunk_ev)));
    for (int64_t e0 = 0; e0 < n_events; e0 += chunk_ev) {
        const int64_t ne = std::min(chunk_ev, n_events - e0);
        const int64_t rows = ne * P;
        hipLaunchKernelGGL(features_kernel, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, st, mom, n_ext,
                           n_events, e0, 1, kap, ne, xev.p, kdev.p);
        hipLaunchKernelGGL(mlp_infer_kernel, dim3(unsigned((rows + FR - 1) / FR)), dim3(256), 0, st, xev.p, P,
                           kap, int(rows), e0, n_events, s->pbf.p, s->par.p, w_in, w_out);
    }
    HIPCHK(hipGetLastError());

    // 2. surrogate sums per point; partial sums, then the audit statistics
    const unsigned sblocks = 256;
    sbuf<double> part(st);
    HIPCHK(part.alloc(size_t(P) * sblocks + size_t(P) * 4));
    double* astats = part.p + size_t(P) * sblocks;
    hipLaunchKernelGGL(sum_rows, dim3(sblocks, unsigned(P)), dim3(256), 0, st, w_out, P, n_events, part.p);

    // 3. audit: events with u(seed, e) < fraction, selected and compacted in
    // event order on the device, evaluated exactly
    const int64_t na = audit_size(seed, audit_fraction, n_events);
    if (na > 0) {
        const int64_t nblk = (n_events + 255) / 256;
        sbuf<unsigned> acount(st);
        sbuf<int64_t> aoff(st), didx(st);
        sbuf<double> mom_a(st), w_a(st), w_ex(st);
        HIPCHK(acount.alloc(size_t(nblk)));
        HIPCHK(aoff.alloc(size_t(nblk) + 1));
        HIPCHK(didx.alloc(size_t(na)));
        HIPCHK(mom_a.alloc(size_t(na) * n_ext * 4));
        HIPCHK(w_a.alloc(size_t(na)));
        HIPCHK(w_ex.alloc(size_t(na) * P));
        hipLaunchKernelGGL(audit_count_kernel, dim3(unsigned(nblk)), dim3(256), 0, st, uint64_t(seed), audit_fraction,
                           n_events, acount.p);
        hipLaunchKernelGGL(audit_scan_kernel, dim3(1), dim3(256), 0, st, acount.p, nblk, aoff.p);
        hipLaunchKernelGGL(audit_fill_kernel, dim3(unsigned(nblk)), dim3(256), 0, st, uint64_t(seed), audit_fraction,
                           n_events, aoff.p, na, didx.p);
        hipLaunchKernelGGL(gather_events, dim3(unsigned((na + 255) / 256)), dim3(256), 0, st, mom, n_ext, n_events,
                           didx.p, na, w_in, mom_a.p, w_a.p);
        r = mgrw_reweight(p, mom_a.p, w_a.p, na, w_ex.p, nullptr, stream);
        if (r != MGRW_OK) return r;
        hipLaunchKernelGGL(audit_kernel, dim3(unsigned(P)), dim3(256), 0, st, didx.p, na, w_ex.p, n_events, w_out,
                           astats);
        HIPCHK(hipGetLastError());
    }
    std::vector<double> host(size_t(P) * sblocks + size_t(P) * 4, 0.0);
    HIPCHK(hipMemcpyAsync(host.data(), part.p, (na > 0 ? host.size() : size_t(P) * sblocks) * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double* stats = host.data() + size_t(P) * sblocks;
    bool bad = false;
    for (int k = 0; k < P; ++k) {
        double ssur = 0.0;
        for (unsigned b = 0; b < sblocks; ++b) ssur += host[size_t(k) * sblocks + b];
        const double d = stats[k * 4], e1 = stats[k * 4 + 1], e2 = stats[k * 4 + 2], m = stats[k * 4 + 3];
        const double mean = m > 0 ? e1 / m : 0.0;
        const double var = m > 1 ? std::max(0.0, (e2 - m * mean * mean) / (m - 1)) : 0.0;
        if (m > 0 && !(mean <= max_audit_error)) bad = true;
        if (audit_stats) {
            audit_stats[k * 5 + 0] = ssur + d / audit_fraction;
            audit_stats[k * 5 + 1] = ssur;
            audit_stats[k * 5 + 2] = mean;
            audit_stats[k * 5 + 3] = m > 0 ? std::sqrt(var / m) : 0.0;
            audit_stats[k * 5 + 4] = double(na);
        }
    }
    if (bad) {   // the audit says the surrogate is not good enough here: exact
        if (fell_back) *fell_back = 1;
        return mgrw_reweight(p, mom, w_in, n_events, w_out, nullptr, stream);
    }
    return MGRW_OK;
}

}  // extern "C"
