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

// ------------------------------------------------------- elementwise kernels

// Feature rows r = e*P + k of events [e0, e0 + rows/P): bfloat16 x[r][64],
// kd[r] = kappa_k - 1.  Features: the 24 momentum components over sqrt(s)/2,
// (kappa - 1)/0.2, then for the 14 particle pairs (i < j) other than the two
// beams v_ij = 2 p_i.p_j / s and log(v_ij); absent particles give zeros.
// The points' kappa values travel by value with each launch.
struct kappa_set {
    double k[MGRW_MAX_POINTS];
};

// nin = 25 keeps only the momentum components and kappa (the invariants'
// columns are zero).
__global__ void features_kernel(const double* __restrict__ mom, int n_ext, int64_t n, int64_t e0, int P,
                                kappa_set kappa, int64_t rows, int nin, uint16_t* __restrict__ x,
                                float* __restrict__ kd) {
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
            xr[c] = nin > c ? f2bf(v) : uint16_t(0);
            xr[c + 14] = nin > c + 14 ? f2bf(lv) : uint16_t(0);
            ++c;
        }
    for (int i = NFEAT; i < K0; ++i) xr[i] = 0;
    kd[r] = float(kappa.k[k] - 1.0);
}

// Feature rows of given float features [m][NFEAT] (tests).
__global__ void features_from_f32(const float* __restrict__ xin, int64_t m, uint16_t* __restrict__ x) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= m) return;
    for (int i = 0; i < K0; ++i) x[r * K0 + i] = i < NFEAT ? f2bf(xin[r * NFEAT + i]) : uint16_t(0);
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
// arithmetic as the training kernels' forward pass.  rows < 2^31.
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

// ------------------------------------------------------------- training
//
// One Adam step on a batch of B sample rows runs in six kernels:
//   train_fwd_kernel  TR rows per workgroup through the four hidden layers
//                     (activations in LDS, as in inference) and the output
//                     unit: loss, dh = d loss / d h, the output layer's
//                     gradient partials and dz4; it stores what the backward
//                     pass needs (a_0..a_3, z_1..z_3, dz4);
//   train_bwd_kernel  per hidden layer l = 4, 3, 2, 1, two kinds of workgroup
//                     in one launch: TR-row tiles of dz_{l-1} = (dz_l W_l) *
//                     SiLU'(z_{l-1}) (l > 1), and
//                     64 x 64 tiles of dW_l = dz_l^T a_{l-1} over one of
//                     kSlices slices of the rows (split-K partials; the tiles
//                     of the first k columns also sum dz_l over the slice:
//                     the bias gradient's partials);
//   adam_kernel       sums the partials, updates the float32 parameters and
//                     refreshes both bfloat16 copies of the weights (row-major
//                     for the forward pass, transposed for dz_l W_l); the
//                     output layer's parameters and the loss, with partials
//                     per row tile, take one wave each.
// Rounding points: features, weights, activations a_l and back-propagated
// dz_l in bfloat16, pre-activations z_l and all accumulation in float32.
// Pre-activations z_l stay float32 and are stored in the order in which the
// lanes of the forward epilogue hold them and the lanes of the dz epilogue
// need them (z_index), so each wave instruction moves 1 KB contiguously.
// The bfloat16 matrices a_l and dz_l live in an 8-row blocked layout: element
// (m, c) of a [rows][C] matrix at ((m / 8) C + c) 8 + m % 8.  Eight
// consecutive rows of one column are then 16 contiguous bytes, which is one
// matrix-core operand register of the weight-gradient product (the reduction
// runs over rows): its operands come straight from L2, without LDS staging.
// Sample order: a keyed bijection of [0, samples) per epoch (a four-round
// Feistel network on the next even power of two, cycle-walking into range).

constexpr int kSlices = 16;   // split-K slices of the weight gradients
constexpr int kFwdWaves = 8;  // waves per forward workgroup
constexpr int kRowAlign = 1024;   // batch buffers are padded to this many rows (4 waves x kSlices x 16)

// offset of layer l's (1..4) weight-gradient partials [kSlices][H][K_l]
__host__ __device__ constexpr int64_t pw_off(int layer) {
    return layer <= 1 ? 0 : int64_t(kSlices) * (int64_t(H) * K0 + int64_t(layer - 2) * H * H);
}
constexpr int64_t kPwFloats = pw_off(5);

struct train_bufs {
    uint16_t* xb;      // a_0 (features), blocked [rows/8][K0][8]
    uint16_t* ab[3];   // a_1..a_3, blocked [rows/8][H][8]
    float* z[3];       // z_1..z_3 in the matrix-core lane order (z_index)
    uint16_t* dzb[2];  // dz_l ping-pong, blocked [rows/8][H][8]: dz4, dz2 in [0]; dz3, dz1 in [1]
    float* pw;         // weight-gradient partials, kPwFloats
    float* pb;         // bias-gradient partials [layer 0..3][kSlices][H]
    float* pw5;        // output-layer partials [row tile][H + 1] (w5, then b5)
    double* ploss;     // loss partials [row tile]
    float* pred;       // predictions [rows]
};

// Where the rows of a batch come from.  P > 1: x holds one feature row per
// event and sample s is event s / P at point s % P (kappa column and kd from
// the point's kappa); P == 1: x and kd hold one row per sample.
struct train_src {
    const uint16_t* x;
    const float* kd;
    const float* y;
    int P;
    kappa_set kappa;
    int64_t ns;        // samples
    uint64_t key;      // permutation key of the epoch
    int shuffle;       // 0: sample i is row i of the sweep
    int hb;            // half width (bits) of the permutation domain, 4^hb >= ns
};

// Offset (in float4) of the four pre-activations a lane holds after a
// layer's product D = W A^T: row tile gt (rows 32 gt ..), unit block ub
// (units 32 ub ..), accumulator group g, lane: units 32 ub + 8 g + 4 (lane /
// 32) .. + 3 of row 32 gt + lane % 32.
__device__ __forceinline__ int64_t z_index(int64_t gt, int ub, int g, int lane) {
    return ((gt * 8 + ub) * 4 + g) * 64 + lane;
}

// The sample at position i of the epoch's order.
__host__ __device__ inline int64_t sample_at(const train_src& S, int64_t i) {
    if (!S.shuffle) return i;
    const uint64_t mask = (uint64_t(1) << S.hb) - 1;
    uint64_t x = uint64_t(i);
    do {
        uint64_t L = x >> S.hb, R = x & mask;
        for (int r = 0; r < 4; ++r) {
            const uint64_t F = smix(S.key + 0x9E3779B97F4A7C15ull * uint64_t(r + 1) + R) & mask;
            const uint64_t T = L ^ F;
            L = R;
            R = T;
        }
        x = (L << S.hb) | R;
    } while (x >= uint64_t(S.ns));
    return int64_t(x);
}

// LDS of the backward kernel: TR = 32 RT rows of dz, or (weight gradient)
// two waves' 64 x 64 float tiles for the reduction over the four waves.
template <int RT>
struct rows_lds {
    union {
        uint16_t act[32 * RT][LDA];
        float red[2 * 64 * 64];
    };
};

// LDS rows [0, TR) x C columns -> blocked layout at global rows r0.. .
template <int TR, int C, int NT = 256>
__device__ __forceinline__ void store_blocked(const uint16_t (*act)[LDA], uint16_t* __restrict__ dst, int r0, int t) {
    constexpr int NB = TR / 8;   // 8-row blocks
    static_assert(C == H || C == K0, "feature or hidden width");
    constexpr int TPC = NT / C;   // threads per column
    const int c = t % C;
    for (int b = t / C; b < NB; b += TPC) {
        uint32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            w[j] = uint32_t(act[b * 8 + 2 * j][c]) | (uint32_t(act[b * 8 + 2 * j + 1][c]) << 16);
        *reinterpret_cast<uint4*>(dst + (int64_t(r0 / 8 + b) * C + c) * 8) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Blocked layout at global rows r0.. -> LDS rows [0, TR) x C columns.
template <int TR, int C, int NT = 256>
__device__ __forceinline__ void load_blocked(const uint16_t* __restrict__ src, uint16_t (*act)[LDA], int r0, int t) {
    constexpr int NB = TR / 8;
    constexpr int TPC = NT / C, NPT = (NB + TPC - 1) / TPC;   // threads per column, blocks per thread
    const int c = t % C, b0 = t / C;
    uint4 v[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i)   // every load first, then the LDS writes
        if (b0 + i * TPC < NB) v[i] = *reinterpret_cast<const uint4*>(src + (int64_t(r0 / 8 + b0 + i * TPC) * C + c) * 8);
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int b = b0 + i * TPC;
        if (b >= NB) break;
        const uint32_t w[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            act[b * 8 + 2 * j][c] = uint16_t(w[j] & 0xffffu);
            act[b * 8 + 2 * j + 1][c] = uint16_t(w[j] >> 16);
        }
    }
}

// Forward pass, loss and output-layer backward of TR = 32 RT rows per
// workgroup (rows b0 + r of the epoch's order) with NW waves, each owning
// UT = 8 / NW tiles of 32 units of every layer; see the section comment.
template <int RT, int NW>
__global__ void __launch_bounds__(64 * NW, 4)
train_fwd_kernel(train_src S, int64_t b0, int rows, double inv_m, const uint16_t* __restrict__ wbf,
                 const float* __restrict__ par, train_bufs T) {
    constexpr int TR = 32 * RT, UT = 8 / NW, NT = 64 * NW;
    __shared__ __align__(16) uint16_t act[TR][LDA];
    __shared__ float kd_s[TR], y_s[TR], dh_s[TR];
    __shared__ double lred[NW];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, lr = lane & 31, lh = lane >> 5;
    const int r0 = int(blockIdx.x) * TR;
    // the weight operands of a whole layer (UT x 16 k-steps of 16 bytes per
    // lane): layer 0's requested first, each next layer's right after the last
    // product of the current one, so that a layer waits for its weights once
    constexpr int KSMAX = H / 16;
    bf16x8 wq[UT][KSMAX];
    auto wload = [&](int l) {
        const int K = K_IN[l];
        const uint16_t* W = wbf + W_OFF[l];   // [H][K]
#pragma unroll
        for (int ut = 0; ut < UT; ++ut)
#pragma unroll
            for (int ks = 0; ks < KSMAX; ++ks)
                if (ks < K / 16)
                    wq[ut][ks] = *reinterpret_cast<const bf16x8*>(W + ((wave * UT + ut) * 32 + lr) * K + ks * 16 + lh * 8);
    };
    wload(0);
    // every load of the prologue is issued before any of them is waited
    // for: biases and output layer (to LDS), the rows' features, kd and y
    __shared__ __align__(16) float pls[4 * H + H + 1];
    constexpr int NPL = (4 * H + H + 1 + NT - 1) / NT;
    float pv[NPL];
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
        const int i = t + j * NT;   // b1..b4 (B_OFF[l] = OFF_B1 + l (H H + H)), then w5, b5
        if (i < 4 * H + H + 1)
            pv[j] = par[i < 4 * H ? OFF_B1 + (i / H) * (int64_t(H) * H + H) + i % H : OFF_W5 + (i - 4 * H)];
    }
    // rows: TR rows, 256 / TR of the first 256 threads per row
    constexpr int TPR = 256 / TR, CPT = K0 / TPR;   // threads per row, feature columns per thread
    const int mrow = t / TPR, q = t % TPR, r = r0 + mrow;
    const bool live = t < 256 && r < rows;
    const bool owner = t < 256 && q == (NRAW - 1) / CPT;   // the thread that copies column 24 of the row
    const int64_t smp = live ? sample_at(S, b0 + r) : 0;
    const uint32_t ev = S.P > 1 ? uint32_t(smp) / uint32_t(S.P) : uint32_t(smp);   // samples < 2^31
    const int pk = S.P > 1 ? int(uint32_t(smp) - ev * uint32_t(S.P)) : 0;
    uint4 xv[CPT / 8];
#pragma unroll
    for (int i = 0; i < CPT / 8; ++i)
        xv[i] = live ? reinterpret_cast<const uint4*>(S.x + int64_t(ev) * K0 + q * CPT)[i] : make_uint4(0u, 0u, 0u, 0u);
    float kd = 0.0f, y = 0.0f;
    if (live && owner) {
        kd = S.P > 1 ? float(S.kappa.k[pk] - 1.0) : S.kd[smp];
        y = S.y[smp];
    }
#pragma unroll
    for (int j = 0; j < NPL; ++j)
        if (t + j * NT < 4 * H + H + 1) pls[t + j * NT] = pv[j];
    if (t < 256) {
#pragma unroll
        for (int i = 0; i < CPT / 8; ++i) reinterpret_cast<uint4*>(&act[mrow][q * CPT])[i] = xv[i];
        if (owner) {
            if (live && S.P > 1) act[mrow][NRAW - 1] = f2bf(float((S.kappa.k[pk] - 1.0) / 0.2));
            kd_s[mrow] = kd;
            y_s[mrow] = y;
        }
    }
    __syncthreads();
    store_blocked<TR, K0, NT>(act, T.xb, r0, t);
    f32x16 acc[UT][RT];   // [unit tile][row tile]; after layer 4: z4
    // the layers unrolled: constant trip counts and offsets let every wait
    // count only the loads it needs
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int KS = K_IN[l] / 16;
#pragma unroll
        for (int ut = 0; ut < UT; ++ut)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[ut][rt] = f32x16{};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8 x[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                x[rt] = *reinterpret_cast<const bf16x8*>(&act[rt * 32 + lr][ks * 16 + lh * 8]);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ut = 0; ut < UT; ++ut)
                    acc[ut][rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq[ut][ks], x[rt], acc[ut][rt], 0, 0, 0);
        }
        if (l < 3) wload(l + 1);
        __syncthreads();   // every wave has read the layer's input
#pragma unroll
        for (int ut = 0; ut < UT; ++ut)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int ub = wave * UT + ut;          // unit block
                const int n = ub * 32 + g * 8 + lh * 4;   // units n .. n+3
                const float4 bn = *reinterpret_cast<const float4*>(&pls[l * H + n]);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    f32x16& c = acc[ut][rt];
                    const float4 z = make_float4(c[4 * g] + bn.x, c[4 * g + 1] + bn.y, c[4 * g + 2] + bn.z,
                                                 c[4 * g + 3] + bn.w);
                    if (l < 3) {
                        reinterpret_cast<float4*>(T.z[l])[z_index(r0 / 32 + rt, ub, g, lane)] = z;
                    } else {   // z4 stays for dz4
                        c[4 * g] = z.x;
                        c[4 * g + 1] = z.y;
                        c[4 * g + 2] = z.z;
                        c[4 * g + 3] = z.w;
                    }
                    *reinterpret_cast<uint2*>(&act[rt * 32 + lr][n]) =
                        make_uint2(pack_bf16(silu(z.x), silu(z.y)), pack_bf16(silu(z.z), silu(z.w)));
                }
            }
        __syncthreads();
        if (l < 3) store_blocked<TR, H, NT>(act, T.ab[l], r0, t);
    }
    // output unit, loss and dh; HPR of the first 256 threads per row
    constexpr int HPR = 256 / TR, UPT = H / HPR;   // threads per row, hidden units per thread
    double lo = 0.0;
    if (t < 256) {
        const int mrow = t / HPR, q = t % HPR, r = r0 + mrow;
        const bool live = r < rows;
        float h = 0.0f;
        const uint4* ar = reinterpret_cast<const uint4*>(&act[mrow][q * UPT]);
        const float4* w5h = reinterpret_cast<const float4*>(&pls[4 * H + q * UPT]);
#pragma unroll
        for (int j = 0; j < UPT / 8; ++j) {
            const uint4 a8 = ar[j];
            const float4 wa = w5h[2 * j], wb = w5h[2 * j + 1];
            h += __uint_as_float(a8.x << 16) * wa.x + __uint_as_float(a8.x & 0xffff0000u) * wa.y;
            h += __uint_as_float(a8.y << 16) * wa.z + __uint_as_float(a8.y & 0xffff0000u) * wa.w;
            h += __uint_as_float(a8.z << 16) * wb.x + __uint_as_float(a8.z & 0xffff0000u) * wb.y;
            h += __uint_as_float(a8.w << 16) * wb.z + __uint_as_float(a8.w & 0xffff0000u) * wb.w;
        }
#pragma unroll
        for (int o = 1; o < HPR; o <<= 1) h += __shfl_xor(h, o);
        h += pls[5 * H];
        const float kr = kd_s[mrow];
        const float yh = kr * h;
        const float diff = yh - y_s[mrow];
        if (q == 0) {
            const float dh = live ? float(2.0 * double(diff) * inv_m) * kr : 0.0f;
            dh_s[mrow] = dh;
            if (live) {
                T.pred[r] = yh;
                lo = double(diff) * double(diff) * inv_m;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lo += __shfl_xor(lo, o, 64);
    if (lane == 0) lred[wave] = lo;
    __syncthreads();
    if (t < 256) {
        // output-layer gradient partials of the tile: dw5[n] = sum dh a4[n], db5 = sum dh
        float sw = 0.0f;
        for (int m = 0; m < TR; ++m) sw += dh_s[m] * bf2f(act[m][t]);
        T.pw5[int64_t(blockIdx.x) * (H + 1) + t] = sw;
        if (t == 0) {
            float sb = 0.0f;
            for (int m = 0; m < TR; ++m) sb += dh_s[m];
            T.pw5[int64_t(blockIdx.x) * (H + 1) + H] = sb;
            double sl = 0.0;
            for (int w = 0; w < NW; ++w) sl += lred[w];
            T.ploss[blockIdx.x] = sl;
        }
    }
    __syncthreads();   // a4 is read; dz4 replaces it
#pragma unroll
    for (int ut = 0; ut < UT; ++ut)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int n = (wave * UT + ut) * 32 + g * 8 + lh * 4;
            const float4 w5 = *reinterpret_cast<const float4*>(&pls[4 * H + n]);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const f32x16& c = acc[ut][rt];
                const float dh = dh_s[rt * 32 + lr];
                *reinterpret_cast<uint2*>(&act[rt * 32 + lr][n]) =
                    make_uint2(pack_bf16(dh * w5.x * dsilu(c[4 * g]), dh * w5.y * dsilu(c[4 * g + 1])),
                               pack_bf16(dh * w5.z * dsilu(c[4 * g + 2]), dh * w5.w * dsilu(c[4 * g + 3])));
            }
        }
    __syncthreads();
    store_blocked<TR, H, NT>(act, T.dzb[0], r0, t);
}

// Backward through hidden layer `layer` (1..4): blocks [0, n_da) form
// dz_{layer-1} for TR-row tiles (layer > 1), the others the weight-gradient
// partials of one 64 x 64 tile and one slice of the rows.  rows_pad: the
// batch rounded up to kRowAlign (each of the slice's four waves takes
// rows_pad / (4 kSlices) rows).
template <int RT, int KIN, bool DA>
__global__ void __launch_bounds__(256, 2)
train_bwd_kernel(int layer, int rows, int rows_pad, int n_da, const uint16_t* __restrict__ wt, train_bufs T) {
    constexpr int TR = 32 * RT;
    __shared__ __align__(16) rows_lds<RT> L;
    uint16_t (*act)[LDA] = L.act;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, lr = lane & 31, lh = lane >> 5;
    const uint16_t* __restrict__ dz = T.dzb[(4 - layer) & 1];
    if constexpr (DA) {
        if (int(blockIdx.x) < n_da) {
            const int r0 = int(blockIdx.x) * TR;
            // the pre-activations z_{layer-1} of this lane's (unit, row)
            // pairs, requested first: they arrive while the product runs
            const float4* __restrict__ zb = reinterpret_cast<const float4*>(T.z[layer - 2]);
            float4 zv[2][4][RT];
#pragma unroll
            for (int ut = 0; ut < 2; ++ut)
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) zv[ut][g][rt] = zb[z_index(r0 / 32 + rt, wave * 2 + ut, g, lane)];
            load_blocked<TR, H>(dz, act, r0, t);   // dz_layer rows r0.. into row-major LDS
            __syncthreads();
            // D[k][m] = sum_n W[n][k] dz[m][n]: the transposed weights (row k
            // contiguous in n) as the first operand, dz rows as the second
            f32x16 acc[2][RT];
#pragma unroll
            for (int ut = 0; ut < 2; ++ut)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[ut][rt] = f32x16{};
#pragma unroll 2
            for (int ks = 0; ks < H / 16; ++ks) {
                bf16x8 w[2], x[RT];
#pragma unroll
                for (int ut = 0; ut < 2; ++ut)
                    w[ut] = *reinterpret_cast<const bf16x8*>(wt + ((wave * 2 + ut) * 32 + lr) * H + ks * 16 + lh * 8);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    x[rt] = *reinterpret_cast<const bf16x8*>(&act[rt * 32 + lr][ks * 16 + lh * 8]);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int ut = 0; ut < 2; ++ut)
                        acc[ut][rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[ut], x[rt], acc[ut][rt], 0, 0, 0);
            }
            __syncthreads();   // every wave has read dz_layer
#pragma unroll
            for (int ut = 0; ut < 2; ++ut)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int k = (wave * 2 + ut) * 32 + g * 8 + lh * 4;   // units k .. k+3 of layer-1
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        const f32x16& c = acc[ut][rt];
                        const float4 z = zv[ut][g][rt];
                        *reinterpret_cast<uint2*>(&act[rt * 32 + lr][k]) =
                            make_uint2(pack_bf16(c[4 * g] * dsilu(z.x), c[4 * g + 1] * dsilu(z.y)),
                                       pack_bf16(c[4 * g + 2] * dsilu(z.z), c[4 * g + 3] * dsilu(z.w)));
                    }
                }
            __syncthreads();
            store_blocked<TR, H>(act, T.dzb[1 - ((4 - layer) & 1)], r0, t);
            return;
        }
    }
    // weight gradient dW[n][k] = sum_m dz[m][n] a[m][k] of a 64 x 64 tile over
    // one slice of the rows; the four waves take consecutive quarters of it
    constexpr int KT = KIN / 64;
    const int b = int(blockIdx.x) - (DA ? n_da : 0);
    const int tile = b % (4 * KT), slice = b / (4 * KT);
    const int n0 = (tile / KT) * 64, k0 = (tile % KT) * 64;
    const int R = rows_pad / (4 * kSlices);   // rows per wave, a multiple of 16
    const int m_begin = (slice * 4 + wave) * R;
    // rows of the batch only (beyond it dz is zero or never written); the
    // last 16-row step may cover dead rows of the last row tile (dz = 0)
    const int m_end = min(m_begin + R, rows);
    const uint16_t* __restrict__ a = layer == 1 ? T.xb : T.ab[layer - 2];
    const bool bias = k0 == 0;   // these tiles also sum dz over the slice
    f32x16 acc[2][2];
    float cs[2] = {0.0f, 0.0f};   // column sums of dz, units n0 + ut 32 + lr, this lane's rows
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{};
    // operands of 16-row steps, kPrefetch steps in flight
    constexpr int kPrefetch = 2;
    bf16x8 A[kPrefetch][2], B[kPrefetch][2];
    auto load = [&](int st, int m) {
        const int64_t mb = (m >> 3) + lh;   // this lane's 8-row block
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
            A[st][ut] = *reinterpret_cast<const bf16x8*>(dz + (mb * H + n0 + ut * 32 + lr) * 8);
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
            B[st][kt] = *reinterpret_cast<const bf16x8*>(a + (mb * KIN + k0 + kt * 32 + lr) * 8);
    };
#pragma unroll
    for (int st = 0; st < kPrefetch; ++st)
        if (m_begin + 16 * st < m_end) load(st, m_begin + 16 * st);
    for (int m = m_begin; m < m_end; m += 16 * kPrefetch) {
#pragma unroll
        for (int st = 0; st < kPrefetch; ++st) {
            if (m + 16 * st >= m_end) break;
#pragma unroll
            for (int ut = 0; ut < 2; ++ut)
#pragma unroll
                for (int kt = 0; kt < 2; ++kt)
                    acc[ut][kt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[st][ut], B[st][kt], acc[ut][kt], 0, 0, 0);
            if (bias) {
#pragma unroll
                for (int ut = 0; ut < 2; ++ut)
#pragma unroll
                    for (int j = 0; j < 8; ++j) cs[ut] += float(A[st][ut][j]);
            }
            const int mn = m + 16 * (st + kPrefetch);
            if (mn < m_end) load(st, mn);
        }
    }
    if (bias) {
        __shared__ float bred[4][64];
#pragma unroll
        for (int ut = 0; ut < 2; ++ut) {
            const float v = cs[ut] + __shfl_xor(cs[ut], 32);   // both 8-row halves
            if (lh == 0) bred[wave][ut * 32 + lr] = v;
        }
        __syncthreads();
        if (t < 64)
            T.pb[(int64_t(layer - 1) * kSlices + slice) * H + n0 + t] =
                (bred[0][t] + bred[1][t]) + (bred[2][t] + bred[3][t]);
    }
    // sum of the four waves' tiles: waves 2, 3 hand theirs to waves 0, 1
    // through LDS, then wave 1 to wave 0, which writes the slice's partial
    float* red = L.red;   // [2][64][64]
    auto tile_pass = [&](int slot, bool add) {
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int nl = ut * 32 + (r / 4) * 8 + lh * 4 + r % 4, kl = kt * 32 + lr;
                    float& x = red[(slot * 64 + nl) * 64 + kl];
                    if (add)
                        acc[ut][kt][r] += x;
                    else
                        x = acc[ut][kt][r];
                }
    };
    if (wave >= 2) tile_pass(wave - 2, false);
    __syncthreads();
    if (wave < 2) tile_pass(wave, true);
    __syncthreads();
    if (wave == 1) tile_pass(0, false);
    __syncthreads();
    if (wave == 0) {
        tile_pass(0, true);
        float* out = T.pw + pw_off(layer) + (int64_t(slice) * H + n0) * KIN + k0;
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int nl = ut * 32 + (r / 4) * 8 + lh * 4 + r % 4, kl = kt * 32 + lr;
                    out[int64_t(nl) * KIN + kl] = acc[ut][kt][r];
                }
    }
}

// Adam on one parameter with gradient g (float32 master, bfloat16 copy).
__device__ __forceinline__ float adam_update(float* __restrict__ p, float* __restrict__ m1, float* __restrict__ m2,
                                             uint16_t* __restrict__ pbf, int64_t i, float g, float lr, float b1,
                                             float b2, float eps, float c1, float c2) {
    const float a = b1 * m1[i] + (1.0f - b1) * g;
    const float b = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = b;
    const float v = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    p[i] = v;
    pbf[i] = f2bf(v);
    return v;
}

// Sum the gradient partials of one step; mode 0: Adam on the float32
// parameters, refreshing the row-major and transposed bfloat16 weights, and
// the step's loss added to *loss; mode 1: the gradient into grad and the loss
// into *loss, parameters untouched.  Blocks [0, n_hidden): one thread per
// hidden-layer parameter (kSlices partials each); then one wave per
// output-layer parameter (w5, b5) and one for the loss, whose partials come
// one per row tile (`tiles` of them).
__global__ void __launch_bounds__(256)
adam_kernel(float* __restrict__ p, float* __restrict__ m1, float* __restrict__ m2, uint16_t* __restrict__ pbf,
            uint16_t* __restrict__ pbft, train_bufs T, int tiles, int n_hidden, int mode, float lr, float b1,
            float b2, float eps, float c1, float c2, float* __restrict__ grad, double* __restrict__ loss) {
    if (int(blockIdx.x) >= n_hidden) {
        const int wv = (int(blockIdx.x) - n_hidden) * 4 + int(threadIdx.x >> 6), lane = threadIdx.x & 63;
        if (wv <= H) {   // w5[wv] or (wv == H) b5
            float g = 0.0f;
            for (int q = lane; q < tiles; q += 64) g += T.pw5[int64_t(q) * (H + 1) + wv];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o, 64);
            if (lane == 0) {
                if (mode == 1)
                    grad[OFF_W5 + wv] = g;
                else
                    adam_update(p, m1, m2, pbf, OFF_W5 + wv, g, lr, b1, b2, eps, c1, c2);
            }
        } else if (wv == H + 1) {
            double sl = 0.0;
            for (int q = lane; q < tiles; q += 64) sl += T.ploss[q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) sl += __shfl_xor(sl, o, 64);
            if (lane == 0) *loss = (mode == 0 ? *loss : 0.0) + sl;
        }
        return;
    }
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= OFF_W5) return;
    int l = 3;
    while (i < W_OFF[l]) --l;
    float g = 0.0f;
    const bool weight = i < B_OFF[l];
    const int64_t wj = i - W_OFF[l];   // index within W_l
    if (weight) {
        const int64_t len = int64_t(H) * K_IN[l];
        const float* pw = T.pw + pw_off(l + 1) + wj;
#pragma unroll
        for (int sl = 0; sl < kSlices; ++sl) g += pw[sl * len];
    } else {
        const float* pb = T.pb + int64_t(l) * kSlices * H + (i - B_OFF[l]);
#pragma unroll
        for (int sl = 0; sl < kSlices; ++sl) g += pb[sl * H];
    }
    if (mode == 1) {
        grad[i] = g;
        return;
    }
    const float v = adam_update(p, m1, m2, pbf, i, g, lr, b1, b2, eps, c1, c2);
    if (weight && l >= 1) {   // W_l[n][k] -> Wt_l[k][n] (layers 2..4)
        const int64_t n = wj / H, k = wj % H;
        pbft[int64_t(l - 1) * H * H + k * H + n] = f2bf(v);
    }
}

// Both bfloat16 copies of freshly set parameters.
__global__ void to_bf16(const float* __restrict__ p, uint16_t* __restrict__ pbf, uint16_t* __restrict__ pbft) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    const uint16_t vb = f2bf(p[i]);
    pbf[i] = vb;
    for (int l = 1; l < 4; ++l)
        if (i >= W_OFF[l] && i < B_OFF[l]) {
            const int64_t wj = i - W_OFF[l], n = wj / H, k = wj % H;
            pbft[int64_t(l - 1) * H * H + k * H + n] = vb;
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
    dbuf<uint16_t> pbf, pbft;   // bfloat16 weights: row-major, and W2..W4 transposed
    // one batch (see train_bufs)
    dbuf<uint16_t> xb, ab[3], dzb[2];
    dbuf<float> z[3], pw, pb, pw5, pred;
    dbuf<double> ploss, lossd;
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

// Rows of the batch buffers for a batch of `rows` (padded to kRowAlign).
int64_t padded_rows(int64_t rows) { return (rows + kRowAlign - 1) / kRowAlign * kRowAlign; }

hipError_t ensure_rows(surrogate* s, int64_t rows) {
    const int64_t rc = padded_rows(rows);
    if (rc <= s->rows_cap) return hipSuccess;
    const int64_t tiles = rc / 32;   // row tiles of the smallest size
    hipError_t e;
    auto zero = [&](auto& b, size_t count) {
        if ((e = b.alloc(count)) != hipSuccess) return false;
        if ((e = hipMemset(b.p, 0, count * sizeof(*b.p))) != hipSuccess) return false;
        return true;
    };
    if (!zero(s->xb, size_t(rc) * K0)) return e;
    for (int l = 0; l < 3; ++l) {
        if (!zero(s->ab[l], size_t(rc) * H)) return e;
        if (!zero(s->z[l], size_t(rc) * H)) return e;
    }
    for (int l = 0; l < 2; ++l)
        if (!zero(s->dzb[l], size_t(rc) * H)) return e;
    if (!zero(s->pw, size_t(kPwFloats))) return e;
    if (!zero(s->pb, size_t(4) * kSlices * H)) return e;
    if (!zero(s->pw5, size_t(tiles) * (H + 1))) return e;
    if (!zero(s->pred, size_t(rc))) return e;
    if (!zero(s->ploss, size_t(tiles))) return e;
    s->rows_cap = rc;
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
    HIPCHK(s->pbft.alloc(size_t(3) * H * H));
    HIPCHK(s->lossd.alloc(1));
    return MGRW_OK;
}

// nin: input features in use (the fan-in of the first layer; the weights of
// unused input columns are zero).
void init_params(std::vector<float>& w, uint64_t seed, int nin = NFEAT) {
    w.assign(NPAR, 0.0f);
    int64_t i = 0;
    auto fill = [&](int64_t off, int rows, int cols, int used_cols, double scale) {
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c)
                w[off + int64_t(r) * cols + c] =
                    c < used_cols ? float((2.0 * u01(seed, 3, uint64_t(i++)) - 1.0) * scale) : 0.0f;
    };
    fill(OFF_W1, H, K0, nin, std::sqrt(6.0 / nin));
    fill(OFF_W2, H, H, H, std::sqrt(6.0 / H));
    fill(OFF_W3, H, H, H, std::sqrt(6.0 / H));
    fill(OFF_W4, H, H, H, std::sqrt(6.0 / H));
    fill(OFF_W5, 1, H, H, 0.1 / std::sqrt(double(H)));
}

train_bufs bufs_of(surrogate* s) {
    train_bufs T;
    T.xb = s->xb.p;
    for (int l = 0; l < 3; ++l) {
        T.ab[l] = s->ab[l].p;
        T.z[l] = s->z[l].p;
    }
    T.dzb[0] = s->dzb[0].p;
    T.dzb[1] = s->dzb[1].p;
    T.pw = s->pw.p;
    T.pb = s->pb.p;
    T.pw5 = s->pw5.p;
    T.ploss = s->ploss.p;
    T.pred = s->pred.p;
    return T;
}

template <int RT>
void launch_step(surrogate* s, const train_src& S, int64_t b0, int rows, hipStream_t st) {
    constexpr int TR = 32 * RT;
    const train_bufs T = bufs_of(s);
    const int tiles = (rows + TR - 1) / TR;
    const int rp = int(padded_rows(rows));
    hipLaunchKernelGGL((train_fwd_kernel<RT, kFwdWaves>), dim3(unsigned(tiles)), dim3(64 * kFwdWaves), 0, st, S, b0,
                       rows, 1.0 / double(rows), s->pbf.p, s->par.p, T);
    for (int layer = 4; layer >= 2; --layer)
        hipLaunchKernelGGL((train_bwd_kernel<RT, H, true>), dim3(unsigned(tiles + 16 * kSlices)), dim3(256), 0, st,
                           layer, rows, rp, tiles, s->pbft.p + size_t(layer - 2) * H * H, T);
    hipLaunchKernelGGL((train_bwd_kernel<RT, K0, false>), dim3(unsigned(4 * kSlices)), dim3(256), 0, st, 1, rows, rp,
                       0, static_cast<const uint16_t*>(nullptr), T);
}

// Row tiles of 32 rows: the most workgroups for a batch (the row-tile
// kernels' time is one workgroup's latency once they all run at once).
constexpr int kRT = 1;
int step_tiles(int rows) { return (rows + 32 * kRT - 1) / (32 * kRT); }

// Forward, backward and (mode 0) Adam for the batch at positions b0 .. b0 +
// rows - 1 of the epoch's order; mode 1 writes the gradient to s->grad and
// the loss to s->lossd instead of updating.
void train_step(surrogate* s, const train_src& S, int64_t b0, int rows, int mode, float lr, hipStream_t st) {
    launch_step<kRT>(s, S, b0, rows, st);
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.0f, c2 = 1.0f;
    if (mode == 0) {
        s->step += 1;
        c1 = 1.0f - std::pow(b1, float(s->step));
        c2 = 1.0f - std::pow(b2, float(s->step));
    }
    const int n_hidden = int((OFF_W5 + 255) / 256), n_out = (H + 2 + 3) / 4;   // w5, b5, loss: one wave each
    hipLaunchKernelGGL(adam_kernel, dim3(unsigned(n_hidden + n_out)), dim3(256), 0, st, s->par.p, s->m1.p, s->m2.p,
                       s->pbf.p, s->pbft.p, bufs_of(s), step_tiles(rows), n_hidden, mode, lr, b1, b2, 1e-8f, c1, c2,
                       s->grad.p, s->lossd.p);
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

// Fit a freshly initialised network (seeded) to the samples of S (their
// order shuffled per epoch by S's permutation); per-epoch mean loss into
// loss_out (host, may be NULL).
mgrw_status train_core(mgrw_process* p, train_src S, const mgrw_train_config* cfg, double* loss_out,
                       hipStream_t st, int nin = NFEAT) {
    std::vector<float> w0;
    init_params(w0, cfg->seed, nin);
    mgrw_status r = mgrw_surrogate_set(p, w0.data());
    if (r != MGRW_OK) return r;
    surrogate* s = p->sur;
    const int64_t B = cfg->batch;
    HIPCHK(ensure_rows(s, B));
    const int64_t nb = S.ns / B;
    if (nb < 1) return set_error(MGRW_ERR_ARG, "fewer samples than one batch");
    S.shuffle = 1;
    S.hb = 1;
    while ((int64_t(1) << (2 * S.hb)) < S.ns) ++S.hb;
    float lr = float(cfg->lr);
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        S.key = smix(cfg->seed + 7919 * uint64_t(ep + 1));
        HIPCHK(hipMemsetAsync(s->lossd.p, 0, sizeof(double), st));
        for (int64_t b = 0; b < nb; ++b) train_step(s, S, b * B, int(B), 0, lr, st);
        HIPCHK(hipGetLastError());
        double lsum = 0.0;
        HIPCHK(hipMemcpyAsync(&lsum, s->lossd.p, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (loss_out) loss_out[ep] = lsum / double(nb);
        lr *= float(cfg->lr_decay);
    }
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
    hipLaunchKernelGGL(to_bf16, dim3(unsigned((NPAR + 255) / 256)), dim3(256), 0, 0, s->par.p, s->pbf.p, s->pbft.p);
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
    sbuf<uint16_t> xall(st);
    HIPCHK(xall.alloc(size_t(m) * K0));
    hipLaunchKernelGGL(features_from_f32, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, x, m, xall.p);
    train_src S{};
    S.x = xall.p;
    S.kd = kd;
    S.y = y;
    S.P = 1;
    S.ns = m;
    S.shuffle = 0;
    train_step(s, S, 0, int(m), 1, 0.0f, st);
    HIPCHK(hipGetLastError());
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

    // labels y = log(W'/W) from the exact kernels (sample s = e P + k): the
    // kappa-polynomial evaluation where the process has it (exact up to
    // rounding, one amplitude program per helicity for all points), else the
    // point-by-point one; the features once per event (the kappa column is
    // set per sample in training)
    sbuf<double> wex(st);
    HIPCHK(wex.alloc(size_t(ns)));
    mgrw_status r = p->proc == MGRW_GG_TTGGG ? mgrw_reweight(p, mom, nullptr, n_events, wex.p, nullptr, stream)
                                             : mgrw_reweight_kpoly(p, mom, nullptr, n_events, wex.p, nullptr, stream);
    if (r != MGRW_OK) return r;
    sbuf<float> yall(st), kdev(st);
    sbuf<uint16_t> xev(st);
    HIPCHK(yall.alloc(size_t(ns)));
    HIPCHK(kdev.alloc(size_t(n_events)));
    HIPCHK(xev.alloc(size_t(n_events) * K0));
    hipLaunchKernelGGL(labels_kernel, dim3(unsigned((ns + 255) / 256)), dim3(256), 0, st, wex.p, P, n_events, yall.p);
    hipLaunchKernelGGL(features_kernel, dim3(unsigned((n_events + 255) / 256)), dim3(256), 0, st, mom, n_ext,
                       n_events, int64_t(0), 1, kappas_of(p), n_events, p->sur_inputs, xev.p, kdev.p);
    HIPCHK(hipGetLastError());
    train_src S{};
    S.x = xev.p;
    S.y = yall.p;
    S.P = P;
    S.kappa = kappas_of(p);
    S.ns = ns;
    return train_core(p, S, cfg, loss_out, st, p->sur_inputs);
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
    sbuf<uint16_t> xall(st);
    HIPCHK(xall.alloc(size_t(m) * K0));
    hipLaunchKernelGGL(features_from_f32, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, x, m, xall.p);
    HIPCHK(hipGetLastError());
    train_src S{};
    S.x = xall.p;
    S.kd = kd;
    S.y = y;
    S.P = 1;
    S.ns = m;
    return train_core(p, S, cfg, loss_out, st);
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
                           n_events, e0, 1, kap, ne, p->sur_inputs, xev.p, kdev.p);
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
