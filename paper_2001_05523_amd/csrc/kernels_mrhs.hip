// Products with many right-hand sides (blocks of RB columns): the panel
// products become small GEMMs.  Vectors are stored row-major per block, entry
// (i, r) at i * RB + r, so that every input segment is a contiguous
// seg_len x RB tile.
//
//   k_rowpanel_mrhs       Y[rows of g] (+)= P_g X[columns of g], FMA in FP64/FP32
//   k_rowpanel_mrhs_mfma  the same on matrix cores: FP32 (16x16x4) or BF16
//                         (16x16x32) inputs with FP32 accumulation
//   k_colpanel_mrhs       transposed product over column panels
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"

namespace h2b {

namespace {

constexpr int NT = 256;

template <typename T> struct AccM { using type = double; };
template <> struct AccM<float> { using type = float; };
template <> struct AccM<bf16_t> { using type = float; };


// Segment descriptors of a group (column offset and input row of every
// segment), held in LDS for groups of up to MSEG segments and read from
// global memory otherwise.
constexpr int MSEG = 128;
struct SegMap {
    const int32_t *c0, *in;
    int n;
    // input row of panel column c: binary search for the last segment with
    // c0 <= c (a zero-length segment shares its start with the next one)
    __device__ int row(int c) const
    {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (c0[mid] <= c)
                lo = mid;
            else
                hi = mid - 1;
        }
        return in[lo] + (c - c0[lo]);
    }
};

// Loads the descriptors of group g into the LDS arrays (all threads of the
// block call it; it ends with a barrier).
__device__ inline SegMap load_segments(const RowPanelDev &d, int g, int32_t *lc0, int32_t *lin)
{
    const int s0 = d.seg_ptr[g], n = d.seg_ptr[g + 1] - s0;
    SegMap m{d.seg_c0 + s0, d.seg_in + s0, n};
    if (n <= MSEG) {
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            lc0[e] = m.c0[e];
            lin[e] = m.in[e];
        }
        m.c0 = lc0;
        m.in = lin;
    }
    __syncthreads();
    return m;
}

// Thread (t) owns rows 4*(t/16) .. +3 (64 rows per pass) and RB/16 right-hand
// sides starting at (t%16)*(RB/16).
template <typename VT, typename XT, typename YT, int ROLE, int RB>
__global__ __launch_bounds__(NT) void k_rowpanel_mrhs(RowPanelDev d, int g0, const VT *__restrict__ vals,
                                                      const XT *__restrict__ x, YT *__restrict__ y,
                                                      int accumulate)
{
    using A = typename AccM<VT>::type;
    constexpr int KC = 32;
    constexpr int CR = RB / 16;
    __shared__ A Ps[64][KC + 1];
    __shared__ A Xs[KC][RB];
    __shared__ int32_t lc0[MSEG], lin[MSEG];
    const int g = g0 + blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const SegMap segs = load_segments(d, g, lc0, lin);
    const int t = threadIdx.x;
    const int rq = (t / 16) * 4, cq = (t % 16) * CR;
    for (int r0 = 0; r0 < nr; r0 += 64) {
        A acc[4][CR];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < CR; ++j) acc[i][j] = 0;
        for (int c0 = 0; c0 < nc; c0 += KC) {
            const int cl = min(KC, nc - c0);
#pragma unroll
            for (int e = t; e < 64 * KC; e += NT) {
                const int i = e / KC, k = e % KC;
                Ps[i][k] = (r0 + i < nr && k < cl) ? (A)vals[off + (int64_t)(r0 + i) * nc + c0 + k] : A(0);
            }
#pragma unroll
            for (int e = t; e < KC * RB; e += NT) {
                const int k = e / RB, r = e % RB;
                Xs[k][r] = (k < cl) ? (A)x[(int64_t)segs.row(c0 + k) * RB + r] : A(0);
            }
            __syncthreads();
#pragma unroll 8
            for (int k = 0; k < KC; ++k) {
                A a[4], b[CR];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = Ps[rq + i][k];
#pragma unroll
                for (int j = 0; j < CR; ++j) b[j] = Xs[k][cq + j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < CR; ++j) acc[i][j] += a[i] * b[j];
            }
            __syncthreads();
        }
        const int ob = d.out_begin[g];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = r0 + rq + i;
            if (row >= nr) continue;
#pragma unroll
            for (int j = 0; j < CR; ++j) {
                YT *dst = y + (int64_t)(ob + row) * RB + cq + j;
                *dst = accumulate ? (YT)((A)*dst + acc[i][j]) : (YT)acc[i][j];
            }
        }
    }
}

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef __bf16 mb8 __attribute__((ext_vector_type(8)));

// Matrix-core version.  The next chunk of panel columns and input rows is
// fetched into registers while the current one is multiplied from LDS.
// Wave w computes the 16x16 output tiles (row tile,
// rhs tile) with index w, w+4, ... among the 4 x (RB/16) tiles of a 64-row
// pass.  FP32: v_mfma_f32_16x16x4f32, lane l holds A[l%16][l/16] and
// B[l/16][l%16].  BF16: v_mfma_f32_16x16x32_bf16, lane l holds
// A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16].  Both return D[4(l/16)+j][l%16].
template <typename VT, int ROLE, int RB, int KC>
__global__ __launch_bounds__(NT) void k_rowpanel_mrhs_mfma(RowPanelDev d, int g0, const VT *__restrict__ vals,
                                                           const float *__restrict__ x, float *__restrict__ y,
                                                           int accumulate)
{
    constexpr bool BF = std::is_same<VT, bf16_t>::value;
    constexpr int KS = BF ? 32 : 4;  // k per instruction
    static_assert(KC % KS == 0, "chunk must be a multiple of the instruction depth");
    constexpr int TILES = 4 * (RB / 16);
    constexpr int TPW = (TILES + 3) / 4;
    constexpr int EA = 64 * KC / NT, EB = KC * RB / NT;  // staged elements per thread
    using S = typename std::conditional<BF, bf16_t, float>::type;
    __shared__ S As[64][KC + (BF ? 8 : 1)];
    __shared__ S Bs[KC][RB + (BF ? 8 : 1)];
    __shared__ int32_t lc0[MSEG], lin[MSEG];
    const int g = g0 + blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const SegMap segs = load_segments(d, g, lc0, lin);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane % 16, lk = lane / 16;
    for (int r0 = 0; r0 < nr; r0 += 64) {
        const int rt = min(64, nr - r0);  // rows of this pass
        // next chunk's panel and input entries, fetched into registers while
        // the current chunk is multiplied
        S ra[EA], rb[EB];
        auto fetch = [&](int c0) {
            const int cl = min(KC, nc - c0);
#pragma unroll
            for (int q = 0; q < EA; ++q) {
                const int e = t + q * NT, i = e / KC, k = e % KC;
                ra[q] = (i < rt && k < cl) ? (S)vals[off + (int64_t)(r0 + i) * nc + c0 + k] : (S)0.f;
            }
#pragma unroll
            for (int q = 0; q < EB; ++q) {
                const int e = t + q * NT, k = e / RB, r = e % RB;
                rb[q] = (k < cl) ? (S)x[(int64_t)segs.row(c0 + k) * RB + r] : (S)0.f;
            }
        };
        mf4 acc[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = mf4{0.f, 0.f, 0.f, 0.f};
        fetch(0);
        for (int c0 = 0; c0 < nc; c0 += KC) {
#pragma unroll
            for (int q = 0; q < EA; ++q) {
                const int e = t + q * NT;
                As[e / KC][e % KC] = ra[q];
            }
#pragma unroll
            for (int q = 0; q < EB; ++q) {
                const int e = t + q * NT;
                Bs[e / RB][e % RB] = rb[q];
            }
            __syncthreads();
            if (c0 + KC < nc) fetch(c0 + KC);
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const int tile = wave + 4 * q;
                if (tile >= TILES) break;
                const int ti = (tile % 4) * 16, tj = (tile / 4) * 16;
                if (ti >= rt) continue;
#pragma unroll
                for (int k0 = 0; k0 < KC; k0 += KS) {
                    if constexpr (BF) {
                        mb8 a, b;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            a[e] = As[ti + li][k0 + 8 * lk + e];
                            b[e] = Bs[k0 + 8 * lk + e][tj + li];
                        }
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
                    } else {
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[ti + li][k0 + lk], Bs[k0 + lk][tj + li],
                                                                      acc[q], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
        const int ob = d.out_begin[g];
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave + 4 * q;
            if (tile >= TILES) break;
            const int ti = (tile % 4) * 16, tj = (tile / 4) * 16;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = r0 + ti + 4 * lk + j;
                if (row >= nr) continue;
                float *dst = y + (int64_t)(ob + row) * RB + tj + li;
                *dst = accumulate ? *dst + acc[q][j] : acc[q][j];
            }
        }
    }
}

typedef double md4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
// 16x16x4 matrix instructions: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// (both types) and receives D[row(l/16, j)][l%16], j < 4: rows 4(l/16)+j for
// FP32 and (l/16)+4j for FP64 (checked on the device with an in-bounds probe).
template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> {
    using type = mf4;
    __device__ static type mma(float a, float b, type c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int j) { return 4 * q + j; }
};
template <> struct MfmaAcc<double> {
    using type = md4;
    __device__ static type mma(double a, double b, type c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int q, int j) { return q + 4 * j; }
};

constexpr int SK_CHUNK = 2048;  // panel columns whose input rows are looked up per pass

// Y[rows of g] (+)= P_g X[columns of g] on matrix cores (16x16x4, FP32 or
// FP64), for groups of at most 64 rows.  The four waves split the columns
// (16 at a time, wave w taking blocks w, w+4, ...) and read both operands
// straight from memory: within a block, lane (i, q) = (l % 16, l / 16) takes
// columns 4q .. 4q+3 in four steps, for the panel entry of row i and for the
// input row of those columns at right-hand side i, so every step is one
// matrix instruction per 16x16 output tile with no staging through LDS.  The
// input row of every column is looked up once per group (binary search over
// the segment descriptors) into LDS.  The four partial tiles are summed in
// LDS at the end, in a fixed order.
template <typename T, int RB>
__global__ __launch_bounds__(NT) void k_panel_mfma(RowPanelDev d, int g0, const T *__restrict__ vals,
                                                   const T *__restrict__ x, T *__restrict__ y, int accumulate)
{
    using M = MfmaAcc<T>;
    using V = typename M::type;
    constexpr int CT = RB / 16;
    __shared__ int32_t lc0[MSEG], lin[MSEG];
    __shared__ int32_t rowidx[SK_CHUNK];
    __shared__ T red[2][4][CT][4][64];  // two waves' partial tiles
    const int g = g0 + blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    if (nr == 0) return;  // uniform over the block
    const int64_t off = d.val_off[g];
    const SegMap segs = load_segments(d, g, lc0, lin);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane % 16, lq = lane / 16;
    const int nrt = (nr + 15) / 16;  // row tiles (<= 4)
    V acc[4][CT];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) acc[a][b] = V{0, 0, 0, 0};
    for (int c0 = 0; c0 < nc; c0 += SK_CHUNK) {
        const int cl = min(SK_CHUNK, nc - c0);
        for (int c = t; c < cl; c += NT) rowidx[c] = segs.row(c0 + c);
        __syncthreads();
        for (int kb = 16 * wave; kb < cl; kb += 64) {
            T av[4][4], bv[CT][4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kb + 4 * lq + j;
                const bool kin = k < cl;
                const int kc = kin ? k : cl - 1;
                const T *xr = x + (int64_t)rowidx[kc] * RB + li;
#pragma unroll
                for (int b = 0; b < CT; ++b) bv[b][j] = kin ? xr[16 * b] : T(0);
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int r = min(16 * a + li, nr - 1);
                    av[a][j] = (a < nrt && kin) ? vals[off + (int64_t)r * nc + c0 + kc] : T(0);
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    if (a >= nrt) continue;
#pragma unroll
                    for (int b = 0; b < CT; ++b) acc[a][b] = M::mma(av[a][j], bv[b][j], acc[a][b]);
                }
        }
        __syncthreads();
    }
    // partial tiles: waves 2, 3 -> LDS, waves 0, 1 add; wave 1 -> LDS, wave 0 adds
    if (wave >= 2)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) red[wave - 2][a][b][j][lane] = acc[a][b][j];
    __syncthreads();
    if (wave < 2)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[a][b][j] += red[wave][a][b][j][lane];
    __syncthreads();
    if (wave == 1)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) red[0][a][b][j][lane] = acc[a][b][j];
    __syncthreads();
    if (wave == 0) {
        const int ob = d.out_begin[g];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if (a >= nrt) continue;
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * a + M::row(lq, j);
                    if (row >= nr) continue;
                    const T v = acc[a][b][j] + red[0][a][b][j][lane];
                    T *dst = y + (int64_t)(ob + row) * RB + 16 * b + li;
                    *dst = accumulate ? *dst + v : v;
                }
        }
    }
}

// FP32 version with vector operand loads.  The right-hand sides are dealt to
// the CT = RB/16 column tiles interleaved, tile b taking columns CT*i + b, so
// the lane that supplies column i of every tile loads its CT inputs of an
// input row as one vector, and its CT outputs of a result row are adjacent.
// The panel entries of a full block of 16 columns are loaded as 16 bytes per
// lane: lane (i, q) takes row i, columns 4q .. 4q+3, which feed the four
// steps j of the block (step j pairs column 4q + j with input row 4q + j).
// The last, partial block of a chunk falls back to the element loads.
template <int RB>
__global__ __launch_bounds__(NT) void k_panel_mfma_f32(RowPanelDev d, int g0, const float *__restrict__ vals,
                                                       const float *__restrict__ x, float *__restrict__ y,
                                                       int accumulate)
{
    constexpr int CT = RB / 16;
    __shared__ int32_t lc0[MSEG], lin[MSEG];
    __shared__ int32_t rowidx[SK_CHUNK];
    __shared__ float red[2][4][CT][4][64];  // two waves' partial tiles
    const int g = g0 + blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    if (nr == 0) return;  // uniform over the block
    const int64_t off = d.val_off[g];
    const SegMap segs = load_segments(d, g, lc0, lin);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane % 16, lq = lane / 16;
    const int nrt = (nr + 15) / 16;  // row tiles (<= 4)
    mf4 acc[4][CT];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) acc[a][b] = mf4{0, 0, 0, 0};
    const float *xl = x + CT * li;
    for (int c0 = 0; c0 < nc; c0 += SK_CHUNK) {
        const int cl = min(SK_CHUNK, nc - c0);
        for (int c = t; c < cl; c += NT) rowidx[c] = segs.row(c0 + c);
        __syncthreads();
        for (int kb = 16 * wave; kb < cl; kb += 64) {
            float av[4][4], bv[4][CT];
            if (kb + 16 <= cl) {  // full block (uniform over the wave)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    __builtin_memcpy(bv[j], xl + (int64_t)rowidx[kb + 4 * lq + j] * RB, sizeof(float) * CT);
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int r = min(16 * a + li, nr - 1);
                    if (a < nrt)
                        __builtin_memcpy(av[a], vals + off + (int64_t)r * nc + c0 + kb + 4 * lq, sizeof(float) * 4);
                    else
                        av[a][0] = av[a][1] = av[a][2] = av[a][3] = 0.0f;
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = kb + 4 * lq + j;
                    const bool kin = k < cl;
                    const int kc = kin ? k : cl - 1;
                    const float *xr = xl + (int64_t)rowidx[kc] * RB;
#pragma unroll
                    for (int b = 0; b < CT; ++b) bv[j][b] = kin ? xr[b] : 0.0f;
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int r = min(16 * a + li, nr - 1);
                        av[a][j] = (a < nrt && kin) ? vals[off + (int64_t)r * nc + c0 + kc] : 0.0f;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    if (a >= nrt) continue;
#pragma unroll
                    for (int b = 0; b < CT; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][j], bv[j][b], acc[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // partial tiles: waves 2, 3 -> LDS, waves 0, 1 add; wave 1 -> LDS, wave 0 adds
    if (wave >= 2)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) red[wave - 2][a][b][j][lane] = acc[a][b][j];
    __syncthreads();
    if (wave < 2)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[a][b][j] += red[wave][a][b][j][lane];
    __syncthreads();
    if (wave == 1)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) red[0][a][b][j][lane] = acc[a][b][j];
    __syncthreads();
    if (wave == 0) {
        const int ob = d.out_begin[g];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if (a >= nrt) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 16 * a + 4 * lq + j;  // FP32 16x16x4: lane (i, q) holds rows 4q + j
                if (row >= nr) continue;
                float v[CT], *dst = y + (int64_t)(ob + row) * RB + CT * li;
                if (accumulate) __builtin_memcpy(v, dst, sizeof(float) * CT);
#pragma unroll
                for (int b = 0; b < CT; ++b) {
                    const float s = acc[a][b][j] + red[0][a][b][j][lane];
                    v[b] = accumulate ? v[b] + s : s;
                }
                __builtin_memcpy(dst, v, sizeof(float) * CT);
            }
        }
    }
}

// Transposed product: Y[ob + j][:] (+)= sum_b sum_i P_b[i][c0 + j] X[in_b + i][:],
// 64 outputs rows per pass, rows of the blocks in chunks of KC staged in LDS.
template <typename VT, typename XT, typename YT, int ROLE, int RB>
__global__ __launch_bounds__(NT) void k_colpanel_mrhs(ColPanelDev d, int g0, const VT *__restrict__ vals,
                                                      const XT *__restrict__ x, YT *__restrict__ y,
                                                      int accumulate)
{
    using A = typename AccM<VT>::type;
    constexpr int KC = 32;
    constexpr int CR = RB / 16;
    __shared__ A Ps[KC][64 + 1];
    __shared__ A Xs[KC][RB];
    const int g = g0 + blockIdx.x;
    const int ob = d.out_begin[g], ol = d.out_len[g];
    const int b0 = d.blk_ptr[g], b1 = d.blk_ptr[g + 1];
    const int t = threadIdx.x;
    const int jq = (t / 16) * 4, cq = (t % 16) * CR;
    for (int j0 = 0; j0 < ol; j0 += 64) {
        A acc[4][CR];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < CR; ++j) acc[i][j] = 0;
        for (int b = b0; b < b1; ++b) {
            const int nrb = d.b_nrows[b];
            const int64_t stride = d.b_stride[b];
            const VT *base = vals + d.b_val_off[b] + d.b_c0[b] + j0;
            const XT *xin = x + (int64_t)d.b_in[b] * RB;
            for (int i0 = 0; i0 < nrb; i0 += KC) {
                const int il = min(KC, nrb - i0);
#pragma unroll
                for (int e = t; e < KC * 64; e += NT) {
                    const int i = e / 64, j = e % 64;
                    Ps[i][j] = (i < il && j0 + j < ol) ? (A)base[(int64_t)(i0 + i) * stride + j] : A(0);
                }
    #pragma unroll
            for (int e = t; e < KC * RB; e += NT) {
                    const int i = e / RB, r = e % RB;
                    Xs[i][r] = (i < il) ? (A)xin[(int64_t)(i0 + i) * RB + r] : A(0);
                }
                __syncthreads();
#pragma unroll 8
                for (int i = 0; i < KC; ++i) {
                    A a[4], bb[CR];
#pragma unroll
                    for (int q = 0; q < 4; ++q) a[q] = Ps[i][jq + q];
#pragma unroll
                    for (int q = 0; q < CR; ++q) bb[q] = Xs[i][cq + q];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int p = 0; p < CR; ++p) acc[q][p] += a[q] * bb[p];
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + jq + q;
            if (j >= ol) continue;
#pragma unroll
            for (int p = 0; p < CR; ++p) {
                YT *dst = y + (int64_t)(ob + j) * RB + cq + p;
                *dst = accumulate ? (YT)((A)*dst + acc[q][p]) : (YT)acc[q][p];
            }
        }
    }
}

__global__ void k_gather_mrhs(const int32_t *__restrict__ perm, int64_t n, int nb, int rb,
                              const double *__restrict__ x, int64_t ldx, double *__restrict__ xp)
{
    const int64_t tot = n * rb;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / rb;
        const int r = (int)(e % rb);
        xp[e] = (r < nb) ? x[perm[k] + r * ldx] : 0.0;
    }
}

__global__ void k_scatter_mrhs(const int32_t *__restrict__ perm, int64_t n, int nb, int rb, double alpha,
                               const double *__restrict__ yp, const double *__restrict__ yp2,
                               double *__restrict__ y, int64_t ldy)
{
    const int64_t tot = n * nb;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e % n;
        const int r = (int)(e / n);
        const double v = yp2 ? yp[k * rb + r] + yp2[k * rb + r] : yp[k * rb + r];
        y[perm[k] + r * ldy] += alpha * v;
    }
}

inline void check_rb(int rb)
{
    if (rb != 16 && rb != 32 && rb != 64) fail(H2B_EINVAL, "block width must be 16, 32 or 64");
}

inline int grid_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + NT - 1) / NT, 1), 1 << 20); }

}  // namespace

template <typename VT, typename XT, typename YT>
void launch_rowpanel_mrhs(const RowPanels &rp, int g0, int g1, int rb, const VT *vals, const XT *x, YT *y,
                          bool accumulate, hipStream_t st, Role role)
{
    check_rb(rb);
    if (g1 <= g0) return;
    const int acc = accumulate ? 1 : 0;
#define H2B_RP(R, RBV)                                                                                       \
    hipLaunchKernelGGL((k_rowpanel_mrhs<VT, XT, YT, R, RBV>), dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0, vals, \
                       x, y, acc)
#define H2B_RP_RB(R)                                                                                         \
    if (rb == 16) H2B_RP(R, 16);                                                                             \
    else if (rb == 32) H2B_RP(R, 32);                                                                        \
    else H2B_RP(R, 64);
    switch (role) {
    case Role::Leaf: H2B_RP_RB(0) break;
    case Role::Transfer: H2B_RP_RB(1) break;
    case Role::Coupling: H2B_RP_RB(2) break;
    default: H2B_RP_RB(3) break;
    }
#undef H2B_RP_RB
#undef H2B_RP
    hip_check(hipGetLastError(), "row panel (multi-rhs) launch");
}

template <typename VT>
void launch_rowpanel_mrhs_mfma(const RowPanels &rp, int g0, int g1, int rb, int kc, const VT *vals,
                               const float *x, float *y, bool accumulate, hipStream_t st)
{
    check_rb(rb);
    if (kc != 32 && kc != 64) fail(H2B_EINVAL, "staging depth must be 32 or 64");
    if (g1 <= g0) return;
    const int acc = accumulate ? 1 : 0;
#define H2B_MF(RBV, KCV)                                                                                      \
    hipLaunchKernelGGL((k_rowpanel_mrhs_mfma<VT, 2, RBV, KCV>), dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0,   \
                       vals, x, y, acc)
    if (kc <= 32) {
        if (rb == 16) H2B_MF(16, 32);
        else if (rb == 32) H2B_MF(32, 32);
        else H2B_MF(64, 32);
    } else {
        if (rb == 16) H2B_MF(16, 64);
        else if (rb == 32) H2B_MF(32, 64);
        else H2B_MF(64, 64);
    }
#undef H2B_MF
    hip_check(hipGetLastError(), "row panel (matrix core) launch");
}

template <typename T>
void launch_panel_mfma(const RowPanels &rp, int g0, int g1, int rb, const T *vals, const T *x, T *y,
                       bool accumulate, hipStream_t st)
{
    check_rb(rb);
    if (rp.max_nrows > 64) fail(H2B_EINVAL, "matrix-core panel product needs groups of at most 64 rows");
    if (g1 <= g0) return;
    const int acc = accumulate ? 1 : 0;
    if constexpr (std::is_same<T, float>::value) {
        if (rb == 16)
            hipLaunchKernelGGL(k_panel_mfma_f32<16>, dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0, vals, x, y, acc);
        else if (rb == 32)
            hipLaunchKernelGGL(k_panel_mfma_f32<32>, dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0, vals, x, y, acc);
        else
            hipLaunchKernelGGL(k_panel_mfma_f32<64>, dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0, vals, x, y, acc);
        hip_check(hipGetLastError(), "panel (matrix core, split columns) launch");
        return;
    }
    if (rb == 16)
        hipLaunchKernelGGL((k_panel_mfma<T, 16>), dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0, vals, x, y, acc);
    else if (rb == 32)
        hipLaunchKernelGGL((k_panel_mfma<T, 32>), dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0, vals, x, y, acc);
    else
        hipLaunchKernelGGL((k_panel_mfma<T, 64>), dim3(g1 - g0), dim3(NT), 0, st, rp.dev, g0, vals, x, y, acc);
    hip_check(hipGetLastError(), "panel (matrix core, split columns) launch");
}

template <typename VT, typename XT, typename YT>
void launch_colpanel_mrhs(const ColPanels &cp, int g0, int g1, int rb, const VT *vals, const XT *x, YT *y,
                          bool accumulate, hipStream_t st, Role role)
{
    check_rb(rb);
    if (g1 <= g0) return;
    const int acc = accumulate ? 1 : 0;
#define H2B_CP(R, RBV)                                                                                       \
    hipLaunchKernelGGL((k_colpanel_mrhs<VT, XT, YT, R, RBV>), dim3(g1 - g0), dim3(NT), 0, st, cp.dev, g0, vals, \
                       x, y, acc)
#define H2B_CP_RB(R)                                                                                         \
    if (rb == 16) H2B_CP(R, 16);                                                                             \
    else if (rb == 32) H2B_CP(R, 32);                                                                        \
    else H2B_CP(R, 64);
    switch (role) {
    case Role::Leaf: H2B_CP_RB(0) break;
    case Role::Transfer: H2B_CP_RB(1) break;
    case Role::Coupling: H2B_CP_RB(2) break;
    default: H2B_CP_RB(3) break;
    }
#undef H2B_CP_RB
#undef H2B_CP
    hip_check(hipGetLastError(), "column panel (multi-rhs) launch");
}

void launch_gather_mrhs(const int32_t *perm, int64_t n, int nb, int rb, const double *x, int64_t ldx,
                        double *xp, hipStream_t st)
{
    check_rb(rb);
    if (nb < 1 || nb > rb) fail(H2B_EINVAL, "block holds 1..rb right-hand sides");
    hipLaunchKernelGGL(k_gather_mrhs, dim3(grid_for(n * rb)), dim3(NT), 0, st, perm, n, nb, rb, x, ldx, xp);
    hip_check(hipGetLastError(), "gather launch");
}

void launch_scatter_mrhs(const int32_t *perm, int64_t n, int nb, int rb, double alpha, const double *yp,
                         const double *yp2, double *y, int64_t ldy, hipStream_t st)
{
    check_rb(rb);
    if (nb < 1 || nb > rb) fail(H2B_EINVAL, "block holds 1..rb right-hand sides");
    hipLaunchKernelGGL(k_scatter_mrhs, dim3(grid_for(n * nb)), dim3(NT), 0, st, perm, n, nb, rb, alpha, yp, yp2,
                       y, ldy);
    hip_check(hipGetLastError(), "scatter launch");
}

#define H2B_MRHS_INST(VT, XT, YT)                                                                           \
    template void launch_rowpanel_mrhs<VT, XT, YT>(const RowPanels &, int, int, int, const VT *, const XT *, \
                                                   YT *, bool, hipStream_t, Role);                          \
    template void launch_colpanel_mrhs<VT, XT, YT>(const ColPanels &, int, int, int, const VT *, const XT *, \
                                                   YT *, bool, hipStream_t, Role);
H2B_MRHS_INST(double, double, double)
H2B_MRHS_INST(float, double, float)
H2B_MRHS_INST(float, float, float)
H2B_MRHS_INST(float, float, double)
H2B_MRHS_INST(bf16_t, float, float)
#undef H2B_MRHS_INST
template void launch_panel_mfma<float>(const RowPanels &, int, int, int, const float *, const float *, float *,
                                       bool, hipStream_t);
template void launch_panel_mfma<double>(const RowPanels &, int, int, int, const double *, const double *,
                                        double *, bool, hipStream_t);
template void launch_rowpanel_mrhs_mfma<float>(const RowPanels &, int, int, int, int, const float *, const float *,
                                               float *, bool, hipStream_t);
template void launch_rowpanel_mrhs_mfma<bf16_t>(const RowPanels &, int, int, int, int, const bf16_t *,
                                                const float *, float *, bool, hipStream_t);

}  // namespace h2b
