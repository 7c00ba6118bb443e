// 3D U-Net kernels for the learned correction between SIRT iterations.
//
// Convolutions are implicit GEMMs on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16: A 16x32, B 32x16, FP32 accumulate).  Lane layout
// of that instruction: lane l holds A[l % 16][8 (l / 16) .. +8] and
// B[8 (l / 16) .. +8][l % 16], and receives C[4 (l / 16) + j][l % 16], j < 4.
// Activations are channels-last BF16, so the 8 consecutive K values a lane
// needs (8 channels of one voxel and tap) are one 16-byte load; weights are
// packed [tap][cout][cin] for the same reason.
//
//  * conv3_fwd: M = voxels (64 per wave), N = cout, K = 27 taps x cin.  The
//    data gradient is the same kernel with mirrored taps and swapped channels.
//  * conv3_wgrad: M = cout, N = cin, K = voxels, one tap per wave, partial
//    sums per chunk of voxels combined in a fixed order.
//  * upconv2_*: the 2x2x2 stride-2 transposed convolution as GEMMs over its 8
//    sub-positions.
//  * pooling, ReLU backward, head, loss, Adam and packing are elementwise.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ctrex_internal.h"

namespace ctrex {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

constexpr int NT = 256;   // threads per workgroup (4 waves)
constexpr int MB = 4;     // 16-voxel M blocks per wave (64 voxels)
constexpr int C1_TY = 8, C1_TZ = 4;   // output rows (y) and planes (z) of a one-channel tile

__device__ __forceinline__ float bf2f(u16 v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
__device__ __forceinline__ u16 f2bf(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<u16>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<u16>(u >> 16);
}

// Two floats rounded to nearest-even BF16 and packed (first in the low half).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    bf16x2 v;
    v[0] = static_cast<__bf16>(lo);
    v[1] = static_cast<__bf16>(hi);
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf16x8 load8(const u16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = static_cast<__bf16>(0.0f);
    return z;
}
__device__ __forceinline__ __bf16 as_bf(u16 v) { return __builtin_bit_cast(__bf16, v); }

__device__ __forceinline__ f32x4 mma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct Vox {
    int z, y, x;
};

// (z, y, x) of voxel v; below 2^32 voxels in 32-bit arithmetic (a 32-bit
// division by a register costs a fraction of a 64-bit one).
__device__ __forceinline__ Vox decode(long long v, int H, int W) {
    Vox r;
    if (static_cast<unsigned long long>(v) <= 0xffffffffull) {
        const uint32_t u = static_cast<uint32_t>(v), t = u / static_cast<uint32_t>(W);
        r.x = static_cast<int>(u - t * static_cast<uint32_t>(W));
        const uint32_t zq = t / static_cast<uint32_t>(H);
        r.y = static_cast<int>(t - zq * static_cast<uint32_t>(H));
        r.z = static_cast<int>(zq);
        return r;
    }
    r.x = static_cast<int>(v % W);
    const long long t = v / W;
    r.y = static_cast<int>(t % H);
    r.z = static_cast<int>(t / H);
    return r;
}

template <bool OUT_F32, bool RELU, bool ACC>
__device__ __forceinline__ void store_out(void *out, long long idx, float val) {
    if (RELU) val = fmaxf(val, 0.0f);
    if (OUT_F32) {
        float *o = static_cast<float *>(out) + idx;
        *o = ACC ? *o + val : val;
    } else {
        u16 *o = static_cast<u16 *>(out) + idx;
        *o = ACC ? f2bf(bf2f(*o) + val) : f2bf(val);
    }
}

// Four consecutive channels of one voxel (lane layout of an MFMA product
// formed as weights x inputs): bias added by the caller, then ReLU, rounding
// and one 8-byte (BF16) or 16-byte (FP32) store; `vec` false (a channel slice
// at a stride or offset not a multiple of 4) stores element by element.
template <bool OUT_F32, bool RELU, bool ACC>
__device__ __forceinline__ void store4(void *out, long long o, float (&v)[4], bool vec) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (RELU) v[j] = fmaxf(v[j], 0.0f);
    if (!vec) {
#pragma unroll
        for (int j = 0; j < 4; ++j) store_out<OUT_F32, false, ACC>(out, o + j, v[j]);
    } else if (OUT_F32) {
        float4 *q = reinterpret_cast<float4 *>(static_cast<float *>(out) + o);
        float4 w = make_float4(v[0], v[1], v[2], v[3]);
        if (ACC) {
            const float4 p = *q;
            w = make_float4(p.x + v[0], p.y + v[1], p.z + v[2], p.w + v[3]);
        }
        *q = w;
    } else {
        uint2 *q = reinterpret_cast<uint2 *>(static_cast<u16 *>(out) + o);
        if (ACC) {
            const uint2 p = *q;
            v[0] += __uint_as_float(p.x << 16);
            v[1] += __uint_as_float(p.x & 0xffff0000u);
            v[2] += __uint_as_float(p.y << 16);
            v[3] += __uint_as_float(p.y & 0xffff0000u);
        }
        *q = make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
    }
}

// ------------------------------------------------------------ conv 3x3x3 ----
// One input channel: K = the 27 taps (padded to 32) of one voxel, one K step,
// LDS-tiled: a workgroup stages the 18 x 10 x 6 input
// block around its 16 x 8 x 4 output voxels once (zeros outside the volume),
// and each lane then reads its eight taps of a voxel from LDS at addresses
// fixed for the whole kernel (the rows of a wave differ by a constant),
// instead of gathering the 27 neighbours of every voxel from global memory
// with 64-bit index arithmetic.  Lane (g, r) takes taps 8 g .. 8 g + 7 of
// voxel r of each row; taps 27 .. 31 read a block of zeros.  Wave w owns z
// plane w of the tile (8 rows of 16 voxels).
template <int COUT, bool OUT_F32, bool RELU, bool ACC>
__global__ __launch_bounds__(NT) void conv3_c1_tile_kernel(const u16 *__restrict__ in, int in_cs,
                                                           int in_off, const u16 *__restrict__ wt,
                                                           const float *__restrict__ bias,
                                                           void *out, int out_cs, int out_off,
                                                           int D, int H, int W, int out_vec) {
    constexpr int TY = C1_TY, TZ = C1_TZ, SX = 18, SY = TY + 2, SZ = TZ + 2;
    constexpr int NEL = SX * SY * SZ;         // staged input values
    constexpr int MBW = TY * TZ / (NT / 64);  // rows per wave
    constexpr int NZ = MBW * SX;              // zero block after the tile
    constexpr int NB = COUT / 16;
    static_assert(MBW == TY, "a wave owns one z plane of the tile");
    __shared__ u16 tile[NEL + NZ];

    const int ntx = (W + 15) / 16, nty = (H + TY - 1) / TY;
    int bi = blockIdx.x;
    const int x0 = (bi % ntx) * 16;
    bi /= ntx;
    const int y0 = (bi % nty) * TY, z0 = (bi / nty) * TZ;

    // ---- stage: every load of the thread in flight before the LDS writes
    constexpr int ITER = (NEL + NZ + NT - 1) / NT;
    u16 v[ITER];
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = threadIdx.x + k * NT;
        const int x = i % SX, y = (i / SX) % SY, z = i / (SX * SY);
        const int gx = x0 + x - 1, gy = y0 + y - 1, gz = z0 + z - 1;
        v[k] = 0;
        if (i < NEL && gx >= 0 && gx < W && gy >= 0 && gy < H && gz >= 0 && gz < D)
            v[k] = in[((static_cast<long long>(gz) * H + gy) * W + gx) * in_cs + in_off];
    }
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = threadIdx.x + k * NT;
        if (i < NEL + NZ) tile[i] = v[k];
    }

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    int addr[8];   // this lane's eight taps of row 0
    bf16x8 b[NB];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int tap = 8 * g + e;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        addr[e] = tap < 27 ? ((wave + 1 + dz) * SY + 1 + dy) * SX + r + 1 + dx : NEL + r;
#pragma unroll
        for (int n = 0; n < NB; ++n)
            b[n][e] = tap < 27 ? as_bf(wt[tap * COUT + n * 16 + r]) : static_cast<__bf16>(0.0f);
    }
    float bco[NB][4];
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int j = 0; j < 4; ++j) bco[n][j] = bias ? bias[n * 16 + 4 * g + j] : 0.0f;
    __syncthreads();

    const f32x4 zero = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int gz = z0 + wave, gx = x0 + r;
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
        bf16x8 a;
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = as_bf(tile[addr[e] + m * SX]);
        const int gy = y0 + m;
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const f32x4 acc = mma(b[n], a, zero);
            if (gz >= D || gy >= H || gx >= W) continue;
            float o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = acc[j] + bco[n][j];
            store4<OUT_F32, RELU, ACC>(
                out, ((static_cast<long long>(gz) * H + gy) * W + gx) * out_cs + out_off + n * 16 + 4 * g,
                o, out_vec != 0);
        }
    }
}

// LDS-tiled form for cin >= 16.  A workgroup computes TY x TZ rows of 16
// output voxels (x) and first stages their input, grown by one voxel on every
// side (zeros outside the volume), in LDS: [z][y][8-channel chunk][x], 16
// bytes per element, so the 16 lanes of an MFMA row group read 256 contiguous
// bytes.  Each A fragment of the GEMM is then one LDS read instead of a
// gather through L1/L2 (every input voxel feeds 27 taps); weights come from
// global memory (the same for every wave, so from the cache).  A wave owns
// MBW consecutive y rows of one z plane, so every LDS offset but the lane's
// base is a compile-time constant.  More than 32 input channels are staged
// and contracted 32 at a time (the tile keeps the 32-channel shape and LDS
// size: 64 channels at once would need a 4 x 2 tile, three times as many
// halo voxels per output, and half the workgroups per CU).  Occupancy hints:
// 16 -> 16 runs 4 waves per SIMD in 128 registers; 32 or 64 inputs with at
// most 32 outputs run 3 (the LDS tile admits three workgroups per CU); 64
// outputs with 32 or 64 inputs run 2 (without the hint the 64 -> 64 tile's
// two epilogue forms took just over 256 registers, one wave per SIMD); 16 ->
// 32 takes what its accumulators leave.  Tiles: 8 x 4 rows for 16 -> 16,
// 8 x 2 otherwise (16 -> 32 measured 0.83 -> 0.70 ms as a data gradient at
// 256^3 with 8 x 2, 16 -> 16 0.46 -> 0.49 ms, so each keeps its faster shape).
template <int CIN, int COUT> struct ConvTile {
    static constexpr int TY = 8, TZ = CIN == 16 && COUT == 16 ? 4 : 2;
};

// Second input and output of a convolution over a channel concatenation: input
// channels k >= ksplit are channel k - ksplit of in2 (only read where the
// kernel's CAT parameter is set), output channels co >= nsplit go to channel
// co - nsplit of out2 (nsplit a multiple of 16).  A plain convolution passes
// ksplit = cin, nsplit = cout.  With `gate` set, output channel co of a voxel
// is zeroed where gate[voxel][gate_off + co] <= 0 (or NaN), before the
// activation and accumulation: the ReLU derivative at the forward activation
// whose gradient a data-gradient convolution produces.
struct CatArgs {
    const u16 *in2;
    int in2_cs, in2_off, ksplit;
    void *out2;
    int out2_cs, out2_off, nsplit;
    const u16 *gate;
    int gate_cs, gate_off;
};

// The 1x1x1 head folded into a 16-output ReLU convolution (BF16 output, no
// accumulate, one input tensor): with `out` set, out[v] = x[v] + s_v (b +
// sum_c h[c] a[v][c]), a = the BF16-rounded activations and s_v = scale
// (times mask[v] if given); the activations are stored only if write_act.
struct HeadArgs {
    const float *h, *b, *x, *mask;
    float scale;
    float *out;
    int write_act;
};

template <int CIN, int COUT, bool OUT_F32, bool RELU, bool ACC, bool CAT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    CIN == 16 ? (COUT == 16 ? 4 : 1) : (COUT <= 32 ? 3 : 2)))) void
conv3_tile_kernel(const u16 *__restrict__ in, int in_cs, int in_off, const u16 *__restrict__ wt,
                  const float *__restrict__ bias, void *out, int out_cs, int out_off, int D, int H,
                  int W, int out_vec, CatArgs cat, HeadArgs head) {
    constexpr int TY = ConvTile<CIN, COUT>::TY, TZ = ConvTile<CIN, COUT>::TZ;
    constexpr int CST = CIN < 32 ? CIN : 32;  // channels staged at a time
    constexpr int NH = CIN / CST;             // staging passes
    constexpr int SX = 18, SY = TY + 2, SZ = TZ + 2, NC = CST / 8;
    constexpr int NEL = SZ * SY * NC * SX;   // 16-byte elements
    constexpr int MBW = TY * TZ / (NT / 64);  // rows per wave
    constexpr int NB = COUT / 16;
    static_assert(TY % MBW == 0, "a wave's rows lie in one z plane");
    __shared__ bf16x8 tile[NEL];

    const int ntx = (W + 15) / 16, nty = (H + TY - 1) / TY;
    int bi = blockIdx.x;
    const int x0 = (bi % ntx) * 16;
    bi /= ntx;
    const int y0 = (bi % nty) * TY, z0 = (bi / nty) * TZ;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int row0 = wave * MBW;                 // first row (y + TY z) of this wave
    const int ym0 = row0 % TY, zm = row0 / TY;
    // element of (row ym0, plane zm, chunk 0, x = r), tap (0, 0, 0)
    const int lbase = (((zm + 1) * SY + ym0 + 1) * NC) * SX + r + 1;
    f32x4 acc[MBW][NB];
#pragma unroll
    for (int m = 0; m < MBW; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

#pragma unroll 1
    for (int h = 0; h < NH; ++h) {
        if (h > 0) __syncthreads();   // every wave is done with the previous half
        // ---- stage the input (channel chunk fastest in global memory).  Element
        // e = (row (z, y)) ROWLEN + col, col = x NC + c; the thread stride NT moves
        // col by NT % ROWLEN and the row by NT / ROWLEN, so (y, z, col) are
        // stepped with adds and one wrap each instead of divisions.  A batch
        // of a thread's loads is issued before its LDS writes, so their
        // latencies overlap instead of adding up (a load-then-write loop
        // waited for each load in turn).
        {
            constexpr int ROWLEN = SX * NC, DCOL = NT % ROWLEN, DROW = NT / ROWLEN;
            constexpr int ITER = (NEL + NT - 1) / NT;
            constexpr int STAGE_BATCH = 6;   // loads in flight per thread
            static_assert(DROW < SY, "one y wrap per step");
            int col = threadIdx.x % ROWLEN, row = threadIdx.x / ROWLEN;
            int y = row % SY, z = row / SY;
#pragma unroll
            for (int k0 = 0; k0 < ITER; k0 += STAGE_BATCH) {
                bf16x8 v[STAGE_BATCH];
                int dst[STAGE_BATCH];
#pragma unroll
                for (int j = 0; j < STAGE_BATCH; ++j) {
                    const int k = k0 + j;
                    const int c = col % NC, x = col / NC;   // NC is a power of 2
                    const int gx = x0 + x - 1, gy = y0 + y - 1, gz = z0 + z - 1;
                    const bool in_tile = k < ITER && threadIdx.x + k * NT < NEL;
                    dst[j] = in_tile ? ((z * SY + y) * NC + c) * SX + x : -1;
                    v[j] = zero8();
                    if (in_tile && gx >= 0 && gx < W && gy >= 0 && gy < H && gz >= 0 && gz < D) {
                        const long long q = (static_cast<long long>(gz) * H + gy) * W + gx;
                        const int k = h * CST + 8 * c;   // first input channel of the chunk
                        const u16 *src = in;
                        int scs = in_cs, sch = in_off + k;
                        if (CAT && k >= cat.ksplit) {
                            src = cat.in2;
                            scs = cat.in2_cs;
                            sch = cat.in2_off + k - cat.ksplit;
                        }
                        v[j] = load8(src + q * scs + sch);
                    }
                    col += DCOL;
                    int dy = DROW;
                    if (col >= ROWLEN) {
                        col -= ROWLEN;
                        ++dy;
                    }
                    y += dy;
                    if (y >= SY) {
                        y -= SY;
                        ++z;
                    }
                }
#pragma unroll
                for (int j = 0; j < STAGE_BATCH; ++j)
                    if (dst[j] >= 0) tile[dst[j]] = v[j];
            }
        }
        __syncthreads();

        // this half's weights; the empty asm makes the pointer opaque, so
        // the 27 per-tap addresses are formed inside the loop over halves
        // instead of being hoisted out of it and held in registers
        const u16 *wh = wt + h * CST;
        if (NH > 1) asm volatile("" : "+v"(wh));
        if constexpr (CIN == 16 || NB > 2) {
            // K steps: for 16 channels pairs of taps (lane groups 0, 1 take tap 2p,
            // channel chunks 0, 1; groups 2, 3 tap 2p + 1; tap 27 is zero padding),
            // otherwise one tap and 32 channels per step.  The fragments of step
            // p + 1 are read while the MFMAs of step p run (two register sets; the
            // scheduling barriers keep the compiler from moving the reads after them).
            constexpr int KSTEPS = CIN == 16 ? 14 : 27;
            auto fetch = [&](int p, bf16x8 (&a)[MBW], bf16x8 (&b)[NB]) {
                const int tap = CIN == 16 ? 2 * p + (g >> 1) : p;
                const int c = CIN == 16 ? (g & 1) : g;
                const bool live = tap < 27;
                const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                const int off = lbase + ((dz * SY + dy) * NC + c) * SX + dx;
#pragma unroll
                for (int m = 0; m < MBW; ++m) a[m] = live ? tile[off + m * NC * SX] : zero8();
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    b[n] = live ? load8(wh + (tap * COUT + n * 16 + r) * CIN + 8 * c) : zero8();
            };
            auto step = [&](const bf16x8 (&a)[MBW], const bf16x8 (&b)[NB]) {
#pragma unroll
                for (int m = 0; m < MBW; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n) acc[m][n] = mma(b[n], a[m], acc[m][n]);
            };
            bf16x8 a0[MBW], b0[NB], a1[MBW], b1[NB];
            fetch(0, a0, b0);
#pragma unroll
            for (int p = 0; p < KSTEPS; p += 2) {
                if (p + 1 < KSTEPS) fetch(p + 1, a1, b1);
                __builtin_amdgcn_sched_barrier(0);
                step(a0, b0);
                __builtin_amdgcn_sched_barrier(0);
                if (p + 2 < KSTEPS) fetch(p + 2, a0, b0);
                __builtin_amdgcn_sched_barrier(0);
                if (p + 1 < KSTEPS) step(a1, b1);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            // One tap and 32 channels per K step, blocked over dy: for each
            // (dz, dx) the wave reads each input row of its span (rows
            // ym0 - 1 .. ym0 + MBW) once and multiplies it with the weights
            // of the three dy taps of the output rows it neighbours, so one
            // LDS read feeds up to three MFMA blocks instead of one.  The
            // next row's fragment (and, at the first row of a (dz, dx), the
            // next pair's weights) is read while the current MFMAs run.
            constexpr int NR = MBW + 2, NS = 9 * NR;
            static_assert(NR % 2 == 0, "rows are taken in pairs");
            auto fetch_b = [&](int q, bf16x8 (&b)[3][NB]) {
                const int dz = q / 3 - 1, dx = q % 3 - 1;
#pragma unroll
                for (int dyi = 0; dyi < 3; ++dyi) {
                    const int tap = (dz + 1) * 9 + dyi * 3 + dx + 1;
#pragma unroll
                    for (int n = 0; n < NB; ++n)
                        b[dyi][n] = load8(wh + (tap * COUT + n * 16 + r) * CIN + 8 * g);
                }
            };
            auto fetch_a = [&](int st) {
                const int q = st / NR, ri = st % NR - 1;
                const int dz = q / 3 - 1, dx = q % 3 - 1;
                return tile[lbase + ((dz * SY + ri) * NC + g) * SX + dx];
            };
            auto rows = [&](int st, const bf16x8 &a, const bf16x8 (&b)[3][NB]) {
                const int ri = st % NR - 1;
#pragma unroll
                for (int dyi = 0; dyi < 3; ++dyi) {
                    const int m = ri - (dyi - 1);   // output row fed with tap dy = dyi - 1
                    if (m < 0 || m >= MBW) continue;
#pragma unroll
                    for (int n = 0; n < NB; ++n) acc[m][n] = mma(b[dyi][n], a, acc[m][n]);
                }
            };
            bf16x8 bq[2][3][NB];
            fetch_b(0, bq[0]);
            bf16x8 a0 = fetch_a(0), a1;
#pragma unroll
            for (int st = 0; st < NS; st += 2) {
                const int q = st / NR;
                if (st % NR == 0 && q + 1 < 9) fetch_b(q + 1, bq[(q + 1) & 1]);
                a1 = fetch_a(st + 1);
                __builtin_amdgcn_sched_barrier(0);
                rows(st, a0, bq[q & 1]);
                __builtin_amdgcn_sched_barrier(0);
                if (st + 2 < NS) a0 = fetch_a(st + 2);
                __builtin_amdgcn_sched_barrier(0);
                rows(st + 1, a1, bq[((st + 1) / NR) & 1]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // ---- epilogue.  The products were formed as weights x inputs, so lane
    // (g, r) holds output channels n 16 + 4 g + j (j < 4) of voxel r of each
    // row: bias, ReLU and rounding four at a time, one 8-byte (BF16) or
    // 16-byte (FP32) store per lane and block, 512 or 1024 contiguous bytes
    // per wave (a channel slice at a stride and offset not multiple of 4
    // stores element by element)
    const int gz = z0 + zm, gx = x0 + r;
    if constexpr (COUT == 16 && RELU && !ACC && !OUT_F32 && !CAT) {
        if (head.out) {
            // lane (g, r): channels 4 g .. 4 g + 3 of voxel r of each row; the
            // four lane groups' partial dot products are added in a fixed
            // order across lanes (xor 16, then xor 32)
            float hh[4], bco[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hh[j] = head.h[4 * g + j];
                bco[j] = bias ? bias[4 * g + j] : 0.0f;
            }
            const float hb = head.b[0];
            // lane group g reads x and the mask of rows 2 g, 2 g + 1 (all rows'
            // loads in flight before the stores)
            static_assert(MBW <= 8, "four lane groups, two rows each");
            float xv[2], sv[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int m = (2 * g + k) % MBW, gy = y0 + ym0 + m;
                xv[k] = 0.0f;
                sv[k] = head.scale;
                if (2 * g + k < MBW && gz < D && gy < H && gx < W) {
                    const long long vox = (static_cast<long long>(gz) * H + gy) * W + gx;
                    xv[k] = head.x[vox];
                    if (head.mask) sv[k] = head.scale * head.mask[vox];
                }
            }
#pragma unroll
            for (int m = 0; m < MBW; ++m) {
                const int gy = y0 + ym0 + m;
                float a[4], p = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    a[j] = bf2f(f2bf(fmaxf(acc[m][0][j] + bco[j], 0.0f)));
                    p = fmaf(hh[j], a[j], p);
                }
                p += __shfl_xor(p, 16, 64);
                p += __shfl_xor(p, 32, 64);
                if (gz >= D || gy >= H || gx >= W) continue;
                const long long vox = (static_cast<long long>(gz) * H + gy) * W + gx;
                if (g == (m >> 1)) {   // the lane group that loaded this row's x
                    const int k = m & 1;
                    head.out[vox] = fmaf(sv[k], hb + p, xv[k]);
                }
                if (head.write_act)
                    store4<false, false, false>(out, vox * out_cs + out_off + 4 * g, a,
                                                out_vec != 0);
            }
            return;
        }
    }
#pragma unroll
    for (int n = 0; n < NB; ++n) {
        const int co0 = n * 16 + 4 * g;
        float bco[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bco[j] = bias ? bias[co0 + j] : 0.0f;
        // the block's destination (the same for the whole workgroup)
        const bool second = n * 16 >= cat.nsplit;
        void *dst = second ? cat.out2 : out;
        const int dcs = second ? cat.out2_cs : out_cs;
        const int dch = second ? cat.out2_off + co0 - cat.nsplit : out_off + co0;
        if (!cat.gate) {
#pragma unroll
            for (int m = 0; m < MBW; ++m) {
                const int gy = y0 + ym0 + m;
                if (gz >= D || gy >= H || gx >= W) continue;
                const long long vox = (static_cast<long long>(gz) * H + gy) * W + gx;
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = acc[m][n][j] + bco[j];
                store4<OUT_F32, RELU, ACC>(dst, vox * dcs + dch, v, out_vec != 0);
            }
            continue;
        }
        // the gate's 4 channels of each row (one 8-byte load: stride and
        // offset are multiples of 8); with at most 32 outputs those of all
        // rows of the block are loaded together, so their latencies overlap
        // (the 64-output tiles have no registers to spare for them)
        constexpr int GB = NB <= 2 ? MBW : 1;   // rows per batch of gate loads
#pragma unroll
        for (int m0 = 0; m0 < MBW; m0 += GB) {
            uint2 gv[GB];
#pragma unroll
            for (int k = 0; k < GB; ++k) {
                const int gy = y0 + ym0 + m0 + k;
                gv[k] = make_uint2(0u, 0u);
                if (gz < D && gy < H && gx < W)
                    gv[k] = *reinterpret_cast<const uint2 *>(
                        cat.gate + ((static_cast<long long>(gz) * H + gy) * W + gx) * cat.gate_cs +
                        cat.gate_off + co0);
            }
#pragma unroll
            for (int k = 0; k < GB; ++k) {
                const int m = m0 + k, gy = y0 + ym0 + m;
                if (gz >= D || gy >= H || gx >= W) continue;
                const long long vox = (static_cast<long long>(gz) * H + gy) * W + gx;
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = acc[m][n][j] + bco[j];
                if (!(__uint_as_float(gv[k].x << 16) > 0.0f)) v[0] = 0.0f;
                if (!(__uint_as_float(gv[k].x & 0xffff0000u) > 0.0f)) v[1] = 0.0f;
                if (!(__uint_as_float(gv[k].y << 16) > 0.0f)) v[2] = 0.0f;
                if (!(__uint_as_float(gv[k].y & 0xffff0000u) > 0.0f)) v[3] = 0.0f;
                store4<OUT_F32, RELU, ACC>(dst, vox * dcs + dch, v, out_vec != 0);
            }
        }
    }
}

// Weight gradient for cin, cout in {16, 32} as LDS-tiled GEMMs (wider layers
// run it per 32-channel block):
// dw[tap][co][ci] = sum_v dout[v][co] in[v + tap][ci], M = cout, N = cin,
// K = 32 voxels of one x row.  A unit is a 32 (x) x 4 (y) column of voxels
// over a run of z planes.  The workgroup stages, per plane, the output
// gradient and (in a ring of three) the input planes, each transposed to
// channel-major rows in LDS, so a lane's eight consecutive K values (voxels of
// one channel) are one 16-byte read.  Wave w takes the nine taps with
// dz = w - 1: each input row it reads once, makes the dx = -1, 0, +1
// fragments from it with 16-bit funnel shifts, and multiplies them with the
// output-gradient rows y' - dy, so one LDS read feeds about two MFMAs.  The
// nine taps' sums stay in registers over all the units of the workgroup, which
// writes them once as its partial (summed over workgroups in a fixed order).
// With bias_part set, the workgroup also sums the output gradient per channel
// (the bias gradient) as it stages it: each thread always stages the same 8
// channels, keeps FP64 sums, and the threads' sums are added in a fixed order
// into bias_part[block][bias_off + co] (row stride bias_ld).
constexpr int WG_X = 32, WG_Y = 4, WG_IX = 48, WG_IY = WG_Y + 2, WG_THREADS = 192;

__device__ __forceinline__ uint32_t funnel16(uint32_t hi, uint32_t lo) {
    return __builtin_amdgcn_alignbit(hi, lo, 16);
}

// (16 -> 16 keeps four waves per SIMD with the bias sums: 126 registers)
template <int CIN, int COUT>
__global__ __launch_bounds__(WG_THREADS) __attribute__((amdgpu_waves_per_eu(
    CIN == 16 && COUT == 16 ? 4 : 1))) void wgrad_tile_kernel(
    const u16 *__restrict__ in, int in_cs, int in_off, const u16 *__restrict__ dout, int dout_cs,
    int dout_off, int D, int H, int W, int zseg, int units, float *__restrict__ partial,
    double *__restrict__ bias_part, int bias_ld, int bias_off) {
    constexpr int MBk = COUT / 16, NBk = CIN / 16;
    // the next plane is loaded during this plane's MFMAs, where the extra
    // registers cost no occupancy (all but 16 -> 16, which keeps four waves
    // per SIMD in 128 registers without it)
    constexpr bool PIPE = !(CIN == 16 && COUT == 16);
    // input rows: x' = x + 8 for x in [-8, 40) (the lanes read x in [-2, 34))
    __shared__ __attribute__((aligned(16))) u16 inT[3][CIN][WG_IY][WG_IX];
    __shared__ __attribute__((aligned(16))) u16 dT[COUT][WG_Y][WG_X];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int dz = wave - 1;
    const int tx = (W + WG_X - 1) / WG_X, ty = (H + WG_Y - 1) / WG_Y;
    f32x4 acc[3][3][MBk][NBk];   // [dy + 1][dx + 1]
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int m = 0; m < MBk; ++m)
#pragma unroll
                for (int n = 0; n < NBk; ++n) acc[a][b][m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // Staging is split into loads (all of a thread's elements of one plane
    // in flight at once) and LDS writes, so the load latencies overlap
    // instead of adding up.
    // input plane zi (zeros outside the volume) into ring slot (zi + 3) % 3
    constexpr int NCH_I = CIN / 8, NXS = 36;   // x in [-2, 34)
    constexpr int NEL_I = WG_IY * NXS * NCH_I, IT_I = (NEL_I + WG_THREADS - 1) / WG_THREADS;
    constexpr int NCH_D = COUT / 8;
    constexpr int NEL_D = WG_Y * WG_X * NCH_D, IT_D = (NEL_D + WG_THREADS - 1) / WG_THREADS;
    static_assert(WG_THREADS % NCH_D == 0, "a thread stages the same 8 channels throughout");
    double bsum[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    auto load_in = [&](int zi, int x0, int y0, uint4 (&v)[IT_I]) {
#pragma unroll
        for (int k = 0; k < IT_I; ++k) {
            const int e = threadIdx.x + k * WG_THREADS;
            const int c = e % NCH_I;
            const int t = e / NCH_I;
            const int xs = t % NXS, iy = t / NXS;
            const int gx = x0 + xs - 2, gy = y0 - 1 + iy;
            v[k] = make_uint4(0u, 0u, 0u, 0u);
            if (e < NEL_I && zi >= 0 && zi < D && gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const long long q = (static_cast<long long>(zi) * H + gy) * W + gx;
                v[k] = *reinterpret_cast<const uint4 *>(in + q * in_cs + in_off + 8 * c);
            }
        }
    };
    auto store_in = [&](int zi, const uint4 (&v)[IT_I]) {
        const int slot = (zi + 3) % 3;
#pragma unroll
        for (int k = 0; k < IT_I; ++k) {
            const int e = threadIdx.x + k * WG_THREADS;
            if (e >= NEL_I) continue;
            const int c = e % NCH_I;
            const int t = e / NCH_I;
            const int xs = t % NXS, iy = t / NXS;
            const uint32_t wv[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
            for (int j = 0; j < 8; ++j)
                inT[slot][8 * c + j][iy][xs + 6] = static_cast<u16>(wv[j >> 1] >> (16 * (j & 1)));
        }
    };
    auto load_dout = [&](int z, int x0, int y0, uint4 (&v)[IT_D]) {
#pragma unroll
        for (int k = 0; k < IT_D; ++k) {
            const int e = threadIdx.x + k * WG_THREADS;
            const int c = e % NCH_D;
            const int t = e / NCH_D;
            const int x = t % WG_X, y = t / WG_X;
            const int gx = x0 + x, gy = y0 + y;
            v[k] = make_uint4(0u, 0u, 0u, 0u);
            if (e < NEL_D && gx < W && gy < H) {
                const long long q = (static_cast<long long>(z) * H + gy) * W + gx;
                v[k] = *reinterpret_cast<const uint4 *>(dout + q * dout_cs + dout_off + 8 * c);
            }
        }
    };
    auto store_dout = [&](const uint4 (&v)[IT_D]) {
#pragma unroll
        for (int k = 0; k < IT_D; ++k) {
            const int e = threadIdx.x + k * WG_THREADS;
            if (e >= NEL_D) continue;
            const int c = e % NCH_D;
            const int t = e / NCH_D;
            const int x = t % WG_X, y = t / WG_X;
            const uint32_t wv[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
            for (int j = 0; j < 8; ++j)
                dT[8 * c + j][y][x] = static_cast<u16>(wv[j >> 1] >> (16 * (j & 1)));
        }
    };
    auto stage_in = [&](int zi, int x0, int y0) {
        uint4 v[IT_I];
        load_in(zi, x0, y0, v);
        store_in(zi, v);
    };

    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        int t = u;
        const int x0 = (t % tx) * WG_X;
        t /= tx;
        const int y0 = (t % ty) * WG_Y;
        const int za = (t / ty) * zseg;
        const int zb = za + zseg < D ? za + zseg : D;
        auto add_bias = [&](const uint4 (&vd)[IT_D]) {
            if (!bias_part) return;   // zeros outside the volume
#pragma unroll
            for (int k = 0; k < IT_D; ++k) {
                if (threadIdx.x + k * WG_THREADS >= NEL_D) continue;
                const uint32_t wv[4] = {vd[k].x, vd[k].y, vd[k].z, vd[k].w};
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    bsum[j] += static_cast<double>(
                        __uint_as_float(j & 1 ? wv[j >> 1] & 0xffff0000u : wv[j >> 1] << 16));
            }
        };
        __syncthreads();   // the previous unit's reads are done
        stage_in(za - 1, x0, y0);
        stage_in(za, x0, y0);
        if constexpr (PIPE) {   // plane za + 1 and the output gradient of za
            uint4 vi[IT_I], vd[IT_D];
            load_in(za + 1, x0, y0, vi);
            load_dout(za, x0, y0, vd);
            store_in(za + 1, vi);
            store_dout(vd);
            add_bias(vd);
        }
        for (int z = za; z < zb; ++z) {
            uint4 vi[IT_I], vd[IT_D];
            if constexpr (!PIPE) {
                load_in(z + 1, x0, y0, vi);
                load_dout(z, x0, y0, vd);
                store_in(z + 1, vi);
                store_dout(vd);
                add_bias(vd);
            } else if (z + 1 < zb) {
                // the next plane's loads stay in flight while this plane's
                // MFMAs run; they go to LDS after the barrier below, into the
                // ring slot of plane z - 1
                load_in(z + 2, x0, y0, vi);
                load_dout(z + 1, x0, y0, vd);
            }
            __syncthreads();
            // this wave's input plane z + dz
            const int slot = (z + dz + 3) % 3;
            bf16x8 a[WG_Y][MBk];
#pragma unroll
            for (int y = 0; y < WG_Y; ++y)
#pragma unroll
                for (int m = 0; m < MBk; ++m)
                    a[y][m] = *reinterpret_cast<const bf16x8 *>(&dT[m * 16 + r][y][8 * g]);
#pragma unroll
            for (int iy = 0; iy < WG_IY; ++iy) {
                bf16x8 b[3][NBk];
#pragma unroll
                for (int n = 0; n < NBk; ++n) {
                    const u16 *row = &inT[slot][n * 16 + r][iy][0];
                    // x' = 8 g + 6 .. 8 g + 17: last dword of chunk g, chunk
                    // g + 1, first dword of chunk g + 2
                    const uint32_t p3 = *reinterpret_cast<const uint32_t *>(row + 8 * g + 6);
                    const uint4 c1 = *reinterpret_cast<const uint4 *>(row + 8 * g + 8);
                    const uint32_t n0 = *reinterpret_cast<const uint32_t *>(row + 8 * g + 16);
                    const uint4 lm = make_uint4(funnel16(c1.x, p3), funnel16(c1.y, c1.x),
                                                funnel16(c1.z, c1.y), funnel16(c1.w, c1.z));
                    const uint4 lp = make_uint4(funnel16(c1.y, c1.x), funnel16(c1.z, c1.y),
                                                funnel16(c1.w, c1.z), funnel16(n0, c1.w));
                    b[0][n] = __builtin_bit_cast(bf16x8, lm);
                    b[1][n] = __builtin_bit_cast(bf16x8, c1);
                    b[2][n] = __builtin_bit_cast(bf16x8, lp);
                }
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const int ry = iy - 1 - dy;   // output-gradient row
                    if (ry < 0 || ry >= WG_Y) continue;
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                        for (int m = 0; m < MBk; ++m)
#pragma unroll
                            for (int n = 0; n < NBk; ++n)
                                acc[dy + 1][dx][m][n] = mma(a[ry][m], b[dx][n], acc[dy + 1][dx][m][n]);
                }
            }
            __syncthreads();
            if constexpr (PIPE) {
                if (z + 1 < zb) {
                    store_in(z + 2, vi);
                    store_dout(vd);
                    add_bias(vd);
                }
            }
        }
    }
    // partial[block][tap][co][ci]: lane (g, r) holds co = 16 m + 4 g + j, ci = 16 n + r
    float *dst = partial + static_cast<long long>(blockIdx.x) * 27 * COUT * CIN;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int tap = (dz + 1) * 9 + a * 3 + b;
#pragma unroll
            for (int m = 0; m < MBk; ++m)
#pragma unroll
                for (int n = 0; n < NBk; ++n)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        dst[(tap * COUT + m * 16 + 4 * g + j) * CIN + n * 16 + r] = acc[a][b][m][n][j];
        }
    if (bias_part) {
        // the staging buffers are free: the threads' sums through LDS, added
        // in thread order per channel
        double *red = reinterpret_cast<double *>(&inT[0][0][0][0]);
        static_assert(sizeof(inT) >= sizeof(double) * 8 * WG_THREADS, "room for the sums");
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) red[threadIdx.x * 8 + j] = bsum[j];
        __syncthreads();
        if (static_cast<int>(threadIdx.x) < COUT) {
            const int c = threadIdx.x / 8, j = threadIdx.x % 8;
            double t = 0.0;
            for (int u = c; u < WG_THREADS; u += NCH_D) t += red[u * 8 + j];
            bias_part[static_cast<long long>(blockIdx.x) * bias_ld + bias_off + threadIdx.x] = t;
        }
    }
}

// Weight gradient, cin == 1, LDS-tiled on the forward kernel's 16 x 8 x 4
// tiles: M = cout, N = taps (27 padded to 32, two blocks), K = 32 voxels (two
// rows of a tile plane).  A workgroup takes a run of consecutive tiles; for
// each it stages the 18 x 10 x 6 input block in LDS (zeros outside the
// volume), and wave w takes plane w: per K step a lane reads 8 output-gradient
// values of its channel (voxels x = 8 (g & 1) + e of row 2 s + (g >> 1)) and
// its tap's 8 inputs from LDS.  Voxels outside the volume contribute zero on
// both sides; taps 27 .. 31 read tap 13's inputs and are not stored.  The four
// waves' sums are added in order and written as the workgroup's partial
// [27][cout].
template <int COUT>
__global__ __launch_bounds__(NT) void conv3_wgrad_c1_tile_kernel(
    const u16 *__restrict__ in, int in_cs, int in_off, const u16 *__restrict__ dout, int dout_cs,
    int dout_off, int D, int H, int W, int tiles_per_wg, float *__restrict__ partial) {
    constexpr int TY = C1_TY, TZ = C1_TZ, SX = 18, SY = TY + 2, SZ = TZ + 2;
    constexpr int NEL = SX * SY * SZ;
    constexpr int MBk = COUT / 16, NOUT = 27 * COUT;
    static_assert(TZ == NT / 64, "a wave owns one z plane of the tile");
    static_assert(TY % 2 == 0, "K steps take two rows");
    __shared__ u16 tile[NEL];
    __shared__ float red[NT / 64][NOUT];

    const int ntx = (W + 15) / 16, nty = (H + TY - 1) / TY, ntz = (D + TZ - 1) / TZ;
    const long long ntiles = static_cast<long long>(ntx) * nty * ntz;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int xs = 8 * (g & 1), rs = g >> 1;   // the lane's 8 voxels: x = xs + e of row 2 s + rs
    int boff[2];                                // LDS element of tap n 16 + r, voxel (xs, row 0)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        int tap = n * 16 + r;
        if (tap >= 27) tap = 13;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        boff[n] = ((wave + 1 + dz) * SY + 1 + dy) * SX + xs + 1 + dx;
    }
    f32x4 acc[MBk][2];
#pragma unroll
    for (int m = 0; m < MBk; ++m) acc[m][0] = acc[m][1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    const long long t0 = static_cast<long long>(blockIdx.x) * tiles_per_wg;
    const long long t1 = t0 + tiles_per_wg < ntiles ? t0 + tiles_per_wg : ntiles;
    for (long long t = t0; t < t1; ++t) {
        const int x0 = static_cast<int>(t % ntx) * 16;
        const long long tq = t / ntx;
        const int y0 = static_cast<int>(tq % nty) * TY, z0 = static_cast<int>(tq / nty) * TZ;
        __syncthreads();   // the previous tile's LDS reads are done
        constexpr int ITER = (NEL + NT - 1) / NT;
        u16 v[ITER];
#pragma unroll
        for (int k = 0; k < ITER; ++k) {
            const int i = threadIdx.x + k * NT;
            const int x = i % SX, y = (i / SX) % SY, z = i / (SX * SY);
            const int gx = x0 + x - 1, gy = y0 + y - 1, gz = z0 + z - 1;
            v[k] = 0;
            if (i < NEL && gx >= 0 && gx < W && gy >= 0 && gy < H && gz >= 0 && gz < D)
                v[k] = in[((static_cast<long long>(gz) * H + gy) * W + gx) * in_cs + in_off];
        }
#pragma unroll
        for (int k = 0; k < ITER; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < NEL) tile[i] = v[k];
        }
        __syncthreads();
        const int gz = z0 + wave;
#pragma unroll
        for (int st = 0; st < TY / 2; ++st) {
            const int row = 2 * st + rs, gy = y0 + row;
            bf16x8 a[MBk], b[2];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gx = x0 + xs + e;
                const bool ok = gz < D && gy < H && gx < W;
                const long long vox = ok ? (static_cast<long long>(gz) * H + gy) * W + gx : 0;
#pragma unroll
                for (int m = 0; m < MBk; ++m)
                    a[m][e] = ok ? as_bf(dout[vox * dout_cs + dout_off + m * 16 + r])
                                 : static_cast<__bf16>(0.0f);
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    b[n][e] = ok ? as_bf(tile[boff[n] + row * SX + e]) : static_cast<__bf16>(0.0f);
            }
#pragma unroll
            for (int m = 0; m < MBk; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n) acc[m][n] = mma(a[m], b[n], acc[m][n]);
        }
    }
    // lane (g, r) holds co = m 16 + 4 g + j, tap = n 16 + r
#pragma unroll
    for (int m = 0; m < MBk; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int tap = n * 16 + r;
                if (tap < 27) red[wave][tap * COUT + m * 16 + 4 * g + j] = acc[m][n][j];
            }
    __syncthreads();
    float *dst = partial + static_cast<long long>(blockIdx.x) * NOUT;
    for (int i = threadIdx.x; i < NOUT; i += NT) {
        float sum = red[0][i];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) sum += red[w][i];
        dst[i] = sum;
    }
}

// dw[co][ci][tap] = sum over chunks of partial[c][tap][co][ci] (FP64, fixed order).
// The partials hold a (cout_b x cin_b) block of the gradient, output
// channels co0 + [0, cout_b), input channels ci0 + [0, cin_b), of a layer
// with cout x cin channels.  A block takes OUTB consecutive outputs; its
// threads read them as 16-byte groups of four, OUTB / 4 threads per chunk row
// and NT / (OUTB / 4) slices of the chunks (slice k sums chunks k, k + SL,
// ...; eight rows' loads in flight per thread), then the slices are added in
// order: a fixed order in FP64.  The output count is a multiple of 4 (cout_b
// is a multiple of 16).  Few outputs over many chunks take OUTB = 4 (more
// slices, more blocks), the others 32 (128 contiguous bytes per chunk row).
template <int OUTB>
__global__ __launch_bounds__(NT) void reduce_wgrad_kernel(const float *__restrict__ partial,
                                                          int chunks, int taps, int cout_b,
                                                          int cin_b, int co0, int ci0, int cout,
                                                          int cin, int tap_major_out,
                                                          float *__restrict__ dw) {
    constexpr int TPO = OUTB / 4, SL = NT / TPO;
    __shared__ double red[SL][OUTB];
    const int n = taps * cout_b * cin_b;
    const int q = threadIdx.x % TPO, sl = threadIdx.x / TPO;
    const int i0 = blockIdx.x * OUTB + 4 * q;   // the partial's [tap][co][ci] order
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    if (i0 < n) {
        const float *p = partial + i0;
#pragma unroll 8
        for (int c = sl; c < chunks; c += SL) {
            const float4 v = *reinterpret_cast<const float4 *>(p + static_cast<long long>(c) * n);
            sum[0] += static_cast<double>(v.x);
            sum[1] += static_cast<double>(v.y);
            sum[2] += static_cast<double>(v.z);
            sum[3] += static_cast<double>(v.w);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[sl][4 * q + j] = sum[j];
    __syncthreads();
    const int o = threadIdx.x, i = blockIdx.x * OUTB + o;
    if (o >= OUTB || i >= n) return;
    double t = 0.0;
    for (int k = 0; k < SL; ++k) t += red[k][o];
    const int tap = i / (cout_b * cin_b);
    const int rem = i - tap * cout_b * cin_b;
    const int co = co0 + rem / cin_b, ci = ci0 + rem % cin_b;
    // conv3: master order [co][ci][tap]; upconv: [ci][co][tap]
    const int ox = tap_major_out ? (ci * cout + co) * taps + tap : (co * cin + ci) * taps + tap;
    dw[ox] = static_cast<float>(t);
}

// Sum the chunks' partials of one gradient block into dw (see above).
hipError_t launch_reduce_wgrad(const float *partial, int chunks, int taps, int cout_b, int cin_b,
                               int co0, int ci0, int cout, int cin, int tap_major_out, float *dw,
                               hipStream_t s) {
    const int n = taps * cout_b * cin_b;
    if (n % 4 != 0 || reinterpret_cast<uintptr_t>(partial) % 16 != 0) return hipErrorInvalidValue;
    if (n / 32 < 128)
        hipLaunchKernelGGL(reduce_wgrad_kernel<4>, dim3((n + 3) / 4), dim3(NT), 0, s, partial,
                           chunks, taps, cout_b, cin_b, co0, ci0, cout, cin, tap_major_out, dw);
    else
        hipLaunchKernelGGL(reduce_wgrad_kernel<32>, dim3((n + 31) / 32), dim3(NT), 0, s, partial,
                           chunks, taps, cout_b, cin_b, co0, ci0, cout, cin, tap_major_out, dw);
    return hipGetLastError();
}

// Per-channel sums over voxels: partial[block][c].
__global__ __launch_bounds__(NT) void channel_sum_kernel(const u16 *__restrict__ x, int cs, int off,
                                                         int c, long long nvox,
                                                         double *__restrict__ partial) {
    // thread t reads 8 channels (8 (t % (c / 8)) ..) of one voxel as one
    // 16-byte load, over voxels strided by NT / (c / 8); c is 16, 32 or 64
    __shared__ double red[NT][8];
    const int cg = c / 8, per = NT / cg;
    const int grp = threadIdx.x % cg, lane_v = threadIdx.x / cg;
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const long long stride = static_cast<long long>(gridDim.x) * per;
    for (long long v = static_cast<long long>(blockIdx.x) * per + lane_v; v < nvox; v += stride) {
        const uint4 w = *reinterpret_cast<const uint4 *>(x + v * cs + off + 8 * grp);
        const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 8; ++k)
            s[k] += static_cast<double>(bf2f(static_cast<u16>(wv[k >> 1] >> (16 * (k & 1)))));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = s[k];
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < c) {
        const int g8 = threadIdx.x / 8, k = threadIdx.x % 8;
        double t = 0.0;
        for (int l = 0; l < per; ++l) t += red[l * cg + g8][k];
        partial[static_cast<long long>(blockIdx.x) * c + threadIdx.x] = t;
    }
}

// out[j] = sum_i partial[i * ld + j] for j < cols (FP64, fixed order).
constexpr int RR_THREADS = 1024;   // threads of a row-reduction block

__global__ __launch_bounds__(RR_THREADS) void reduce_rows_kernel(const double *__restrict__ partial,
                                                                 int rows, int cols, int ld,
                                                                 float *__restrict__ out) {
    // 32 columns per block, 32 slices of the rows (eight rows' loads in
    // flight per thread: the sums are short, so latency, not bandwidth,
    // bounds them), the slices added in a fixed order
    constexpr int SL = RR_THREADS / 32;
    __shared__ double red[SL][32];
    const int o = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const int jc = blockIdx.x * 32 + o;
    double sum = 0.0;
    if (jc < cols) {
#pragma unroll 8
        for (int i = sl; i < rows; i += SL) sum += partial[static_cast<long long>(i) * ld + jc];
    }
    red[sl][o] = sum;
    __syncthreads();
    if (sl != 0 || jc >= cols) return;
    double t = 0.0;
    for (int k = 0; k < SL; ++k) t += red[k][o];
    out[jc] = static_cast<float>(t);
}

// ------------------------------------------------------ 2x transposed conv --
// out[2i + a][co] = bias[co] + sum_ci in[i][ci] wt[a][co][ci] for the 8
// sub-positions a.  A wave takes 64 consecutive input voxels, reads their
// channels once, and for each sub-position forms the products as weights x
// inputs, so lane (g, r) holds output channels n 16 + 4 g + j of input voxel
// m 16 + r's child a, stored four at a time.
template <int CIN, int COUT, bool OUT_F32, bool ACC>
__global__ __launch_bounds__(NT) void upconv2_fwd_kernel(const u16 *__restrict__ in, int in_cs,
                                                         int in_off, const u16 *__restrict__ wt,
                                                         const float *__restrict__ bias, void *out,
                                                         int out_cs, int out_off, int D, int H,
                                                         int W, int out_vec) {
    constexpr int NB = COUT / 16, KS = CIN / 32;
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const long long nvox = static_cast<long long>(D) * H * W;
    const long long base = (static_cast<long long>(blockIdx.x) * (NT / 64) + (threadIdx.x >> 6)) * 64;
    if (base >= nvox) return;
    const int H2 = 2 * H, W2 = 2 * W;
    bf16x8 av[KS][MB];
    long long child0[MB];   // output index of child (0, 0, 0) of voxel m 16 + r
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const Vox p = decode(base + m * 16 + r, H, W);
        child0[m] = ((static_cast<long long>(2 * p.z) * H2) + 2 * p.y) * W2 + 2 * p.x;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            av[ks][m] = load8(in + (base + m * 16 + r) * in_cs + in_off + ks * 32 + 8 * g);
    }
    const f32x4 zero = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int a = 0; a < 8; ++a) {
        const long long da = ((static_cast<long long>(a >> 2) * H2) + ((a >> 1) & 1)) * W2 + (a & 1);
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            bf16x8 bv[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                bv[ks] = load8(wt + (a * COUT + n * 16 + r) * CIN + ks * 32 + 8 * g);
            const int co0 = n * 16 + 4 * g;
            float bco[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bco[j] = bias ? bias[co0 + j] : 0.0f;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                f32x4 acc = zero;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) acc = mma(bv[ks], av[ks][m], acc);
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = acc[j] + bco[j];
                store4<OUT_F32, false, ACC>(out, (child0[m] + da) * out_cs + out_off + co0, v,
                                            out_vec != 0);
            }
        }
    }
}

// din[i][ci] = sum_a sum_co dout[2i + a][co] wd[a][ci][co]; K = 8 COUT.
template <int CIN, int COUT, bool ACC>
__global__ __launch_bounds__(NT) void upconv2_dgrad_kernel(const u16 *__restrict__ dout, int dout_cs,
                                                           int dout_off, const u16 *__restrict__ wd,
                                                           u16 *__restrict__ din, int din_cs,
                                                           int din_off, int D, int H, int W) {
    constexpr int NB = CIN / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const long long nvox = static_cast<long long>(D) * H * W;
    const long long base = (static_cast<long long>(blockIdx.x) * (NT / 64) + (threadIdx.x >> 6)) * 64;
    if (base >= nvox) return;
    const int H2 = 2 * H, W2 = 2 * W;
    Vox pa[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) pa[m] = decode(base + m * 16 + r, H, W);
    f32x4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < (8 * COUT) / 32; ++s) {
        const int k0 = s * 32 + 8 * g;
        const int a = k0 / COUT, co = k0 % COUT;
        const int az = a >> 2, ay = (a >> 1) & 1, ax = a & 1;
        bf16x8 av[MB], bv[NB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const long long o = ((static_cast<long long>(2 * pa[m].z + az) * H2) + (2 * pa[m].y + ay)) * W2 +
                                (2 * pa[m].x + ax);
            av[m] = load8(dout + o * dout_cs + dout_off + co);
        }
#pragma unroll
        for (int n = 0; n < NB; ++n) bv[n] = load8(wd + (a * CIN + n * 16 + r) * COUT + co);
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[m][n] = mma(av[m], bv[n], acc[m][n]);
    }
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long long v = base + m * 16 + 4 * g + j;
                store_out<false, false, ACC>(din, v * din_cs + din_off + n * 16 + r, acc[m][n][j]);
            }
}

// dw partial[c][a][co][ci] = sum over the chunk of dout[2i + a][co] in[i][ci]; wave = a.
template <int CIN, int COUT>
__global__ __launch_bounds__(NT) void upconv2_wgrad_kernel(const u16 *__restrict__ in, int in_cs,
                                                           int in_off, const u16 *__restrict__ dout,
                                                           int dout_cs, int dout_off, int D, int H,
                                                           int W, long long chunk,
                                                           float *__restrict__ partial) {
    constexpr int MBk = COUT / 16, NBk = CIN / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int a = blockIdx.y * (NT / 64) + (threadIdx.x >> 6);   // 0..7
    const int az = a >> 2, ay = (a >> 1) & 1, ax = a & 1;
    const int H2 = 2 * H, W2 = 2 * W;
    const long long nvox = static_cast<long long>(D) * H * W;
    const long long v0 = static_cast<long long>(blockIdx.x) * chunk;
    const long long v1 = v0 + chunk < nvox ? v0 + chunk : nvox;
    f32x4 acc[MBk][NBk];
#pragma unroll
    for (int m = 0; m < MBk; ++m)
#pragma unroll
        for (int n = 0; n < NBk; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (long long vk = v0; vk < v1; vk += 32) {
        bf16x8 av[MBk], bv[NBk];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const long long v = vk + 8 * g + e;
            const bool ok = v < v1;
            const Vox p = decode(ok ? v : 0, H, W);
            const long long o = ((static_cast<long long>(2 * p.z + az) * H2) + (2 * p.y + ay)) * W2 +
                                (2 * p.x + ax);
#pragma unroll
            for (int m = 0; m < MBk; ++m)
                av[m][e] = ok ? as_bf(dout[o * dout_cs + dout_off + m * 16 + r])
                              : static_cast<__bf16>(0.0f);
#pragma unroll
            for (int n = 0; n < NBk; ++n)
                bv[n][e] = ok ? as_bf(in[v * in_cs + in_off + n * 16 + r]) : static_cast<__bf16>(0.0f);
        }
#pragma unroll
        for (int m = 0; m < MBk; ++m)
#pragma unroll
            for (int n = 0; n < NBk; ++n) acc[m][n] = mma(av[m], bv[n], acc[m][n]);
    }
    float *dst = partial + (static_cast<long long>(blockIdx.x) * 8 + a) * COUT * CIN;
#pragma unroll
    for (int m = 0; m < MBk; ++m)
#pragma unroll
        for (int n = 0; n < NBk; ++n)
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[(m * 16 + 4 * g + j) * CIN + n * 16 + r] = acc[m][n][j];
}

// ---------------------------------------------------------- elementwise ----
__global__ __launch_bounds__(NT) void maxpool2_kernel(const u16 *__restrict__ in, int in_cs, int in_off,
                                                      int c, u16 *__restrict__ out, int D, int H,
                                                      int W) {
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const long long n = static_cast<long long>(Do) * Ho * Wo * c;
    const long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (i >= n) return;
    const int ch = static_cast<int>(i % c);
    const Vox p = decode(i / c, Ho, Wo);
    float m = -__builtin_inff();
    for (int a = 0; a < 8; ++a) {
        const long long q = (static_cast<long long>(2 * p.z + (a >> 2)) * H + 2 * p.y + ((a >> 1) & 1)) * W +
                            2 * p.x + (a & 1);
        m = fmaxf(m, bf2f(in[q * in_cs + in_off + ch]));
    }
    out[i] = f2bf(m);
}

// The same, 8 channels per thread (16-byte loads and store): channel counts,
// strides and offsets multiples of 8, 16-byte aligned tensors.  Each channel
// takes the same fmaxf sequence as above, so the results are identical.
__global__ __launch_bounds__(NT) void maxpool2_vec8_kernel(const u16 *__restrict__ in, int in_cs,
                                                           int in_off, int c8,
                                                           u16 *__restrict__ out, int D, int H,
                                                           int W) {
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const long long n = static_cast<long long>(Do) * Ho * Wo * c8;
    const long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (i >= n) return;
    const long long pv = i / c8;
    const int ch = 8 * static_cast<int>(i - pv * c8);
    const Vox p = decode(pv, Ho, Wo);
    float m[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) m[j] = -__builtin_inff();
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const long long q = (static_cast<long long>(2 * p.z + (a >> 2)) * H + 2 * p.y + ((a >> 1) & 1)) * W +
                            2 * p.x + (a & 1);
        const uint4 v = *reinterpret_cast<const uint4 *>(in + q * in_cs + in_off + ch);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 8; ++j)
            m[j] = fmaxf(m[j], __uint_as_float(j & 1 ? w[j >> 1] & 0xffff0000u : w[j >> 1] << 16));
    }
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        o[k] = static_cast<uint32_t>(f2bf(m[2 * k])) | (static_cast<uint32_t>(f2bf(m[2 * k + 1])) << 16);
    *reinterpret_cast<uint4 *>(out + pv * (8 * c8) + ch) = make_uint4(o[0], o[1], o[2], o[3]);
}

// RELU: then the ReLU derivative at in, over every input element: din is
// zeroed where in <= 0 (or NaN) and left as it is elsewhere, so only the
// arg-max element's din is read.
template <bool RELU>
__global__ __launch_bounds__(NT) void maxpool2_bwd_kernel(const u16 *__restrict__ in, int in_cs,
                                                          int in_off, int c,
                                                          const u16 *__restrict__ dout,
                                                          u16 *__restrict__ din, int D, int H, int W) {
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const long long n = static_cast<long long>(Do) * Ho * Wo * c;
    const long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (i >= n) return;
    const int ch = static_cast<int>(i % c);
    const Vox p = decode(i / c, Ho, Wo);
    float m = -__builtin_inff();
    long long best = -1;
    bool pos[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const long long q = (static_cast<long long>(2 * p.z + (a >> 2)) * H + 2 * p.y + ((a >> 1) & 1)) * W +
                            2 * p.x + (a & 1);
        const float v = bf2f(in[q * in_cs + in_off + ch]);
        pos[a] = v > 0.0f;
        if (v > m || best < 0) {
            m = v;
            best = q;
        }
    }
    u16 *o = din + best * in_cs + in_off + ch;
    if (!RELU || m > 0.0f) *o = f2bf(bf2f(*o) + bf2f(dout[i]));
    if (RELU) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            if (pos[a]) continue;
            const long long q = (static_cast<long long>(2 * p.z + (a >> 2)) * H + 2 * p.y + ((a >> 1) & 1)) * W +
                                2 * p.x + (a & 1);
            din[q * in_cs + in_off + ch] = 0;
        }
    }
}

__global__ __launch_bounds__(NT) void relu_bwd_kernel(const u16 *__restrict__ y, u16 *__restrict__ gr,
                                                      int cs, int off, int c, long long nvox) {
    const long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (i >= nvox * c) return;
    const long long idx = (i / c) * cs + off + i % c;
    if (!(bf2f(y[idx]) > 0.0f)) gr[idx] = 0;
}

// The same, 8 channels (16 bytes) per thread: channel slices at strides and
// offsets that are multiples of 8 (every U-Net activation).
__global__ __launch_bounds__(NT) void relu_bwd8_kernel(const u16 *__restrict__ y, u16 *__restrict__ gr,
                                                       int cs, int off, int c8, long long n8) {
    const long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (i >= n8) return;
    const long long v = i / c8;
    const long long idx = v * cs + off + 8 * (i - v * c8);
    const uint4 a = *reinterpret_cast<const uint4 *>(y + idx);
    uint4 *gp = reinterpret_cast<uint4 *>(gr + idx);
    uint4 q = *gp;
    // a BF16 value h is > 0 when its sign bit is clear and its magnitude bits
    // lie in (0, 0x7f80] (+0 and NaN are not; +inf is), as in the scalar form
    auto pos = [](uint32_t h) { return (h & 0x8000u) == 0 && h != 0 && h <= 0x7f80u; };
    auto keep = [&](uint32_t w, uint32_t g) {
        const uint32_t lo = pos(w & 0xffffu) ? 0xffffu : 0u;
        const uint32_t hi = pos(w >> 16) ? 0xffff0000u : 0u;
        return g & (lo | hi);
    };
    q = make_uint4(keep(a.x, q.x), keep(a.y, q.y), keep(a.z, q.z), keep(a.w, q.w));
    *gp = q;
}

// out = x + m scale (b + sum_k h_k act_k), m = mask[v] (1 without a mask)
__global__ __launch_bounds__(NT) void head_kernel(const u16 *__restrict__ act, int c,
                                                  const float *__restrict__ h, const float *__restrict__ b,
                                                  const float *__restrict__ x, float scale,
                                                  const float *__restrict__ mask,
                                                  float *__restrict__ out, long long n) {
    const long long v = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (v >= n) return;
    float s = b[0];
    for (int k = 0; k < c; ++k) s = fmaf(h[k], bf2f(act[v * c + k]), s);
    const float sc = mask ? scale * mask[v] : scale;
    out[v] = fmaf(sc, s, x[v]);
}

// The same for C channels (a multiple of 8) read 8 at a time, same order of
// operations (so the same result).
template <int C>
__global__ __launch_bounds__(NT) void head_vec_kernel(const u16 *__restrict__ act,
                                                      const float *__restrict__ h,
                                                      const float *__restrict__ b,
                                                      const float *__restrict__ x, float scale,
                                                      const float *__restrict__ mask,
                                                      float *__restrict__ out, long long n) {
    const long long v = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (v >= n) return;
    const uint4 *ap = reinterpret_cast<const uint4 *>(act + v * C);
    float s = b[0];
#pragma unroll
    for (int q = 0; q < C / 8; ++q) {
        const uint4 a = ap[q];
        const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t bits = k & 1 ? w[k >> 1] & 0xffff0000u : w[k >> 1] << 16;
            s = fmaf(h[8 * q + k], __uint_as_float(bits), s);
        }
    }
    const float sc = mask ? scale * mask[v] : scale;
    out[v] = fmaf(sc, s, x[v]);
}

// xb = BF16(scale x)
__global__ __launch_bounds__(NT) void scale_bf16_kernel(const float *__restrict__ x, float scale,
                                                        u16 *__restrict__ xb, long long n) {
    const long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (i < n) xb[i] = f2bf(scale * x[i]);
}

// With d = mask scale dout: dact = d h (RELU: zero where act <= 0, the
// gradient at the pre-activation); per-block partial sums of d act[:, k]
// (k < C) and d.
template <int C, bool VEC, bool RELU>
__global__ __launch_bounds__(NT) void head_bwd_kernel(const u16 *__restrict__ act,
                                                      const float *__restrict__ h, float scale,
                                                      const float *__restrict__ mask,
                                                      const float *__restrict__ dout,
                                                      u16 *__restrict__ dact, long long n,
                                                      double *__restrict__ partial) {
    __shared__ double red[NT];
    double acc[C + 1];
#pragma unroll
    for (int k = 0; k <= C; ++k) acc[k] = 0.0;
    const long long stride = static_cast<long long>(gridDim.x) * NT;
    static_assert(C % 8 == 0, "8 channels per 16-byte access");
    // a counted loop (unrolled by 4), so several voxels' loads are in flight
    const long long v0 = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    const int iters = v0 < n ? static_cast<int>((n - v0 + stride - 1) / stride) : 0;
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
        const long long v = v0 + it * stride;
        const float d = (mask ? scale * mask[v] : scale) * dout[v];
        if constexpr (!VEC) {   // act or dact not 16-byte aligned
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const float a = bf2f(act[v * C + k]);
                acc[k] += static_cast<double>(d) * a;
                dact[v * C + k] = RELU && !(a > 0.0f) ? 0 : f2bf(d * h[k]);
            }
            acc[C] += d;
            continue;
        }
        const uint4 *ap = reinterpret_cast<const uint4 *>(act + v * C);
        uint4 *dp = reinterpret_cast<uint4 *>(dact + v * C);
#pragma unroll
        for (int q = 0; q < C / 8; ++q) {
            const uint4 a = ap[q];
            const uint32_t w[4] = {a.x, a.y, a.z, a.w};
            uint32_t o[4];
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                const int k = 8 * q + 2 * k2;
                const float a0 = __uint_as_float(w[k2] << 16);
                const float a1 = __uint_as_float(w[k2] & 0xffff0000u);
                acc[k] += static_cast<double>(d) * a0;
                acc[k + 1] += static_cast<double>(d) * a1;
                const uint32_t lo = RELU && !(a0 > 0.0f) ? 0u : f2bf(d * h[k]);
                const uint32_t hi = RELU && !(a1 > 0.0f) ? 0u : f2bf(d * h[k + 1]);
                o[k2] = lo | (hi << 16);
            }
            dp[q] = make_uint4(o[0], o[1], o[2], o[3]);
        }
        acc[C] += d;
    }
#pragma unroll
    for (int k = 0; k <= C; ++k) {
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
            if (static_cast<int>(threadIdx.x) < s2) red[threadIdx.x] += red[threadIdx.x + s2];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[static_cast<long long>(blockIdx.x) * (C + 1) + k] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(NT) void mse_kernel(const float *__restrict__ a, const float *__restrict__ t,
                                                 long long n, float scale, float *__restrict__ grad,
                                                 double *__restrict__ partial) {
    __shared__ double red[NT];
    double s = 0.0;
    const long long stride = static_cast<long long>(gridDim.x) * NT;
    for (long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) {
        const float d = a[i] - t[i];
        s += static_cast<double>(d) * d;
        if (grad) grad[i] = scale * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (static_cast<int>(threadIdx.x) < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void adam_kernel(float *__restrict__ p, const float *__restrict__ gr,
                                                  float *__restrict__ m, float *__restrict__ v,
                                                  long long n, float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
    const long long i = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
    if (i >= n) return;
    const float gv = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gv;
    const float vi = b2 * v[i] + (1.0f - b2) * gv * gv;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// w [cout][cin][taps] -> wt [tap][cout][cin] and wt_d [taps-1-tap][cin][cout] (mirrored)
__global__ __launch_bounds__(NT) void pack_kernel(const float *__restrict__ w, int cout, int cin,
                                                  int taps, int mirror, u16 *__restrict__ wt,
                                                  u16 *__restrict__ wt_d, int in_major) {
    const int n = cout * cin * taps;
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    int co, ci, t;
    if (in_major) {   // upconv master [cin][cout][taps]
        ci = i / (cout * taps);
        const int rem = i - ci * cout * taps;
        co = rem / taps;
        t = rem - co * taps;
    } else {          // conv master [cout][cin][taps]
        co = i / (cin * taps);
        const int rem = i - co * cin * taps;
        ci = rem / taps;
        t = rem - ci * taps;
    }
    const u16 b = f2bf(w[i]);
    if (wt) wt[(t * cout + co) * cin + ci] = b;
    if (wt_d) {
        const int td = mirror ? taps - 1 - t : t;
        wt_d[(td * cin + ci) * cout + co] = b;
    }
}

inline unsigned blocks_for(long long n, int per = NT) {
    return static_cast<unsigned>((n + per - 1) / per);
}

}  // namespace

// ---------------------------------------------------------------- launchers --
// The tiled convolution over a two-tensor concatenation is built for the
// decoder shapes only (the up-sampled features and the skip features, equal
// halves of the input).
template <int CI, int CO> constexpr bool cat_shape() {
    return (CI == 32 && CO == 16) || (CI == 64 && CO == 32);
}

inline bool vec_ok(const void *p, int cs, int off) {
    return cs % 4 == 0 && off % 4 == 0 && reinterpret_cast<uintptr_t>(p) % 16 == 0;
}

template <int CI, int CO, bool F32, bool RELU, bool ACC>
hipError_t conv3_go(hipStream_t s, const u16 *ip, int in_cs, int in_off, const u16 *wp,
                    const float *bias, void *out, int out_cs, int out_off, int D, int H, int W,
                    const CatArgs &cat, const HeadArgs &head) {
    // four channels per store: 4-aligned channel slices of 16-byte aligned tensors
    const int out_vec = vec_ok(out, out_cs, out_off) && vec_ok(cat.out2, cat.out2_cs, cat.out2_off);
    const bool two_in = cat.ksplit < CI;
    if constexpr (CI == 1) {
        if (two_in || cat.nsplit < CO) return hipErrorInvalidValue;
        const long long tiles = static_cast<long long>((W + 15) / 16) * ((H + C1_TY - 1) / C1_TY) *
                                ((D + C1_TZ - 1) / C1_TZ);
        hipLaunchKernelGGL((conv3_c1_tile_kernel<CO, F32, RELU, ACC>),
                           dim3(static_cast<unsigned>(tiles)), dim3(NT), 0, s, ip, in_cs, in_off,
                           wp, bias, out, out_cs, out_off, D, H, W, out_vec);
    } else {
        constexpr int TY = ConvTile<CI, CO>::TY, TZ = ConvTile<CI, CO>::TZ;
        const long long tiles = static_cast<long long>((W + 15) / 16) * ((H + TY - 1) / TY) *
                                ((D + TZ - 1) / TZ);
        const dim3 grid(static_cast<unsigned>(tiles));
        if (two_in) {
            if constexpr (cat_shape<CI, CO>())
                hipLaunchKernelGGL((conv3_tile_kernel<CI, CO, F32, RELU, ACC, true>), grid,
                                   dim3(NT), 0, s, ip, in_cs, in_off, wp, bias, out, out_cs,
                                   out_off, D, H, W, out_vec, cat, head);
            else
                return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((conv3_tile_kernel<CI, CO, F32, RELU, ACC, false>), grid, dim3(NT),
                               0, s, ip, in_cs, in_off, wp, bias, out, out_cs, out_off, D, H, W,
                               out_vec, cat, head);
        }
    }
    return hipGetLastError();
}

template <int CI, int CO>
hipError_t conv3_pick(bool relu, bool acc, bool f32, hipStream_t s, const u16 *ip, int in_cs,
                      int in_off, const u16 *wp, const float *bias, void *out, int out_cs,
                      int out_off, int D, int H, int W, const CatArgs &cat) {
    const int k = (f32 ? 4 : 0) | (relu ? 2 : 0) | (acc ? 1 : 0);
    const HeadArgs head{};   // no head
#define GO(F, R, A) \
    return conv3_go<CI, CO, F, R, A>(s, ip, in_cs, in_off, wp, bias, out, out_cs, out_off, D, H, W, \
                                     cat, head)
    switch (k) {
        case 0: GO(false, false, false);
        case 1: GO(false, false, true);
        case 2: GO(false, true, false);
        case 3: GO(false, true, true);
        case 4: GO(true, false, false);
        case 5: GO(true, false, true);
        case 6: GO(true, true, false);
        default: GO(true, true, true);
    }
#undef GO
}

hipError_t launch_conv3(const void *in, int in_cs, int in_off, int cin_a, const void *in2,
                        int in2_cs, int in2_off, int cin_b, const void *wt, const float *bias,
                        void *out, int out_cs, int out_off, int cout_a, void *out2, int out2_cs,
                        int out2_off, int cout_b, const void *gate, int gate_cs, int gate_off,
                        int D, int H, int W, bool relu, bool acc, bool out_f32, hipStream_t s) {
    const int cin = cin_a + cin_b, cout = cout_a + cout_b;
    const u16 *ip = static_cast<const u16 *>(in);
    const u16 *wp = static_cast<const u16 *>(wt);
    CatArgs cat;
    cat.in2 = cin_b > 0 ? static_cast<const u16 *>(in2) : ip;
    cat.in2_cs = cin_b > 0 ? in2_cs : in_cs;
    cat.in2_off = cin_b > 0 ? in2_off : in_off + cin_a;
    cat.ksplit = cin_a;
    cat.out2 = cout_b > 0 ? out2 : out;
    cat.out2_cs = cout_b > 0 ? out2_cs : out_cs;
    cat.out2_off = cout_b > 0 ? out2_off : out_off + cout_a;
    cat.nsplit = cout_a;
    cat.gate = static_cast<const u16 *>(gate);
    cat.gate_cs = gate_cs;
    cat.gate_off = gate_off;
    if (gate && cin == 1) return hipErrorInvalidValue;
    if (cin_a <= 0 || cout_a <= 0 || cout_a % 16 != 0 || (cin_b > 0 && cin_a % 8 != 0))
        return hipErrorInvalidValue;
#define CASE(CI, CO)                                                                             \
    if (cin == CI && cout == CO)                                                                 \
        return conv3_pick<CI, CO>(relu, acc, out_f32, s, ip, in_cs, in_off, wp, bias, out, out_cs, \
                                  out_off, D, H, W, cat);
    if (cin == 1 && cout == 16)
        return conv3_pick<1, 16>(relu, acc, out_f32, s, ip, in_cs, in_off, wp, bias, out, out_cs,
                                 out_off, D, H, W, cat);
    CASE(16, 16)
    CASE(16, 32)
    CASE(32, 16)
    CASE(32, 32)
    CASE(32, 64)
    CASE(64, 32)
    CASE(64, 64)
#undef CASE
    return hipErrorInvalidValue;
}

// A 16 -> 16 ReLU convolution with the head folded in (see HeadArgs); `act`
// (BF16, channel stride act_cs, offset act_off) receives the activations when
// not NULL.
hipError_t launch_conv3_head(const void *in, int in_cs, int in_off, const void *wt,
                             const float *bias, void *act, int act_cs, int act_off, const float *h,
                             const float *hb, const float *x, float scale, const float *mask,
                             float *out, int D, int H, int W, hipStream_t s) {
    CatArgs cat{};
    cat.ksplit = 16;   // one input tensor
    cat.nsplit = 16;   // one output tensor
    cat.out2 = act;
    cat.out2_cs = act_cs;
    cat.out2_off = act_off;
    HeadArgs head;
    head.h = h;
    head.b = hb;
    head.x = x;
    head.mask = mask;
    head.scale = scale;
    head.out = out;
    head.write_act = act != nullptr;
    return conv3_go<16, 16, false, true, false>(s, static_cast<const u16 *>(in), in_cs, in_off,
                                                static_cast<const u16 *>(wt), bias, act, act_cs,
                                                act_off, D, H, W, cat, head);
}

long long wgrad_chunk(long long nvox) {
    // about 2048 chunks on large volumes, at least 512 voxels each
    long long chunk = (nvox + 2047) / 2048;
    chunk = (chunk + 31) / 32 * 32;
    return chunk < 512 ? 512 : chunk;
}

// One input channel: at most about 8192 partials (chunks of at least 512
// voxels), each the sum of one workgroup's run of tiles; they stay small (27
// cout floats each).
long long wgrad_c1_chunk(long long nvox) {
    long long chunk = (nvox + 8191) / 8192;
    chunk = (chunk + 31) / 32 * 32;
    return chunk < 512 ? 512 : chunk;
}

// Bytes of the weight partials, rounded up to 256 (the bias partials follow).
size_t wgrad_partial_bytes(long long chunks, int cin, int cout) {
    const size_t b = sizeof(float) * static_cast<size_t>(chunks) * 27 * cin * cout;
    return (b + 255) / 256 * 256;
}

size_t conv3_wgrad_scratch(int cin, int cout, long long nvox) {
    const long long ch = cin == 1 ? wgrad_c1_chunk(nvox) : wgrad_chunk(nvox);
    const long long chunks = (nvox + ch - 1) / ch;
    // cin > 1: FP64 bias partials [chunks][cout] after the weight partials
    return wgrad_partial_bytes(chunks, cin, cout) +
           (cin > 1 ? sizeof(double) * static_cast<size_t>(chunks) * cout : 0);
}

hipError_t launch_conv3_wgrad(const void *in, int in_cs, int in_off, int cin_a, const void *in2,
                              int in2_cs, int in2_off, int cin_b, const void *dout, int dout_cs,
                              int dout_off, int cout, int D, int H, int W, float *dw,
                              float *dbias, float *scratch, hipStream_t s) {
    const int cin = cin_a + cin_b;
    const long long nvox = static_cast<long long>(D) * H * W;
    const long long chunk = wgrad_chunk(nvox);
    const int chunks = static_cast<int>((nvox + chunk - 1) / chunk);
    const u16 *ip = static_cast<const u16 *>(in), *dp = static_cast<const u16 *>(dout);
    if (cin == 1) {
        if (cout != 16 || cin_b != 0 || dbias) return hipErrorInvalidValue;
        // at most as many workgroups (partials) as the scratch sizing assumes
        const long long c1 = wgrad_c1_chunk(nvox);
        const long long n1 = (nvox + c1 - 1) / c1;
        const long long ntiles = static_cast<long long>((W + 15) / 16) * ((H + C1_TY - 1) / C1_TY) *
                                 ((D + C1_TZ - 1) / C1_TZ);
        const long long per = (ntiles + n1 - 1) / n1;
        const int wgs = static_cast<int>((ntiles + per - 1) / per);
        hipLaunchKernelGGL((conv3_wgrad_c1_tile_kernel<16>), dim3(wgs), dim3(NT), 0, s, ip, in_cs,
                           in_off, dp, dout_cs, dout_off, D, H, W, static_cast<int>(per), scratch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_reduce_wgrad(scratch, wgs, 27, cout, 1, 0, 0, cout, 1, 0, dw, s);
    }
    const auto chan_ok = [](int c) { return c == 16 || c == 32 || c == 64; };
    if (!chan_ok(cin_a) || (cin_b != 0 && !chan_ok(cin_b)) || cin > 64 || !chan_ok(cout))
        return hipErrorInvalidValue;
    // Units: 32 x 4 voxel columns over runs of z planes, at most `chunks`
    // workgroups (each loops over its units).  The input channels (of one
    // tensor or of a two-tensor concatenation) and 64 output channels are
    // split into blocks of at most 32, each a tiled GEMM of its own writing
    // its partials after the previous block's; the scratch (chunks x 27 x cin
    // x cout floats) holds them all.
    const long long tiles = static_cast<long long>((W + WG_X - 1) / WG_X) * ((H + WG_Y - 1) / WG_Y);
    long long zsegs = chunks / tiles;
    if (zsegs < 1) zsegs = 1;
    if (zsegs > D) zsegs = D;
    const int zseg = static_cast<int>((D + zsegs - 1) / zsegs);
    const long long units = tiles * ((D + zseg - 1) / zseg);
    const int parts = static_cast<int>(units < chunks ? units : chunks);
    const int cob = cout < 32 ? cout : 32;
    struct Source {
        const u16 *p;
        int cs, off, c, ci0;
    };
    const Source src[2] = {{ip, in_cs, in_off, cin_a, 0},
                           {static_cast<const u16 *>(in2), in2_cs, in2_off, cin_b, cin_a}};
    float *part = scratch;
    // bias partials [parts][cout] (FP64) after all weight partials; the first
    // input block of each output block sums its output gradient
    double *bpart = reinterpret_cast<double *>(reinterpret_cast<char *>(scratch) +
                                               wgrad_partial_bytes(parts, cin, cout));
    for (int co0 = 0; co0 < cout; co0 += cob)
        for (const Source &sc : src) {
            const int cib = sc.c < 32 ? sc.c : 32;
            for (int l = 0; l < sc.c; l += cib) {
                double *bp = dbias && &sc == &src[0] && l == 0 ? bpart : nullptr;
#define CTREX_NN_WGT(CI, CO)                                                                      \
                if (cib == CI && cob == CO)                                                       \
                    hipLaunchKernelGGL((wgrad_tile_kernel<CI, CO>), dim3(parts),                  \
                                       dim3(WG_THREADS), 0, s, sc.p, sc.cs, sc.off + l, dp,       \
                                       dout_cs, dout_off + co0, D, H, W, zseg,                    \
                                       static_cast<int>(units), part, bp, cout, co0);
                CTREX_NN_WGT(16, 16)
                CTREX_NN_WGT(16, 32)
                CTREX_NN_WGT(32, 16)
                CTREX_NN_WGT(32, 32)
#undef CTREX_NN_WGT
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                e = launch_reduce_wgrad(part, parts, 27, cob, cib, co0, sc.ci0 + l, cout, cin, 0,
                                        dw, s);
                if (e != hipSuccess) return e;
                part += static_cast<long long>(parts) * 27 * cob * cib;
            }
        }
    if (dbias)
        hipLaunchKernelGGL(reduce_rows_kernel, dim3(blocks_for(cout, 32)), dim3(RR_THREADS), 0, s,
                           bpart, parts, cout, cout, dbias);
    return hipGetLastError();
}

size_t channel_sum_scratch(int c) { return sizeof(double) * 1024 * static_cast<size_t>(c); }

hipError_t launch_channel_sum(const void *x, int cs, int off, int c, long long nvox, float *out,
                              double *scratch, hipStream_t s) {
    if (c % 8 || c < 8 || c > 64) return hipErrorInvalidValue;
    const int blocks = 1024;
    hipLaunchKernelGGL(channel_sum_kernel, dim3(blocks), dim3(NT), 0, s, static_cast<const u16 *>(x),
                       cs, off, c, nvox, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(blocks_for(c, 32)), dim3(RR_THREADS), 0, s,
                       scratch, blocks, c, c, out);
    return hipGetLastError();
}

hipError_t launch_upconv2(const void *in, int in_cs, int in_off, int cin, const void *wt,
                          const float *bias, void *out, int out_cs, int out_off, int cout, int D,
                          int H, int W, bool acc, bool out_f32, hipStream_t s) {
    const long long nvox = static_cast<long long>(D) * H * W;
    const dim3 grid(blocks_for(nvox, NT)), blk(NT);
    const u16 *ip = static_cast<const u16 *>(in), *wp = static_cast<const u16 *>(wt);
    const int ov = (out_cs % 4 == 0 && out_off % 4 == 0 &&
                    reinterpret_cast<uintptr_t>(out) % 16 == 0) ? 1 : 0;
#define CTREX_NN_UP_GO(CI, CO, F, A)                                                              \
    hipLaunchKernelGGL((upconv2_fwd_kernel<CI, CO, F, A>), grid, blk, 0, s, ip, in_cs, in_off, wp, \
                       bias, out, out_cs, out_off, D, H, W, ov)
#define CTREX_NN_UP(CI, CO)                                                                       \
    if (cin == CI && cout == CO) {                                                                \
        if (out_f32) {                                                                            \
            if (acc) CTREX_NN_UP_GO(CI, CO, true, true);                                          \
            else CTREX_NN_UP_GO(CI, CO, true, false);                                             \
        } else {                                                                                  \
            if (acc) CTREX_NN_UP_GO(CI, CO, false, true);                                         \
            else CTREX_NN_UP_GO(CI, CO, false, false);                                            \
        }                                                                                         \
        return hipGetLastError();                                                                 \
    }
    CTREX_NN_UP(64, 32)
    CTREX_NN_UP(32, 16)
    CTREX_NN_UP(32, 32)
    CTREX_NN_UP(64, 64)
#undef CTREX_NN_UP
#undef CTREX_NN_UP_GO
    return hipErrorInvalidValue;
}

hipError_t launch_upconv2_dgrad(const void *dout, int dout_cs, int dout_off, int cout,
                                const void *wd, void *din, int din_cs, int din_off, int cin, int D,
                                int H, int W, bool acc, hipStream_t s) {
    const long long nvox = static_cast<long long>(D) * H * W;
    const dim3 grid(blocks_for(nvox, NT)), blk(NT);
    const u16 *dp = static_cast<const u16 *>(dout), *wp = static_cast<const u16 *>(wd);
    u16 *op = static_cast<u16 *>(din);
#define CTREX_NN_UD(CI, CO)                                                                        \
    if (cin == CI && cout == CO) {                                                                 \
        if (acc) { hipLaunchKernelGGL((upconv2_dgrad_kernel<CI, CO, true>), grid, blk, 0, s, dp, dout_cs, dout_off, wp, op, din_cs, din_off, D, H, W); } \
            else { hipLaunchKernelGGL((upconv2_dgrad_kernel<CI, CO, false>), grid, blk, 0, s, dp, dout_cs, dout_off, wp, op, din_cs, din_off, D, H, W); } \
        return hipGetLastError();                                                                  \
    }
    CTREX_NN_UD(64, 32)
    CTREX_NN_UD(32, 16)
    CTREX_NN_UD(32, 32)
    CTREX_NN_UD(64, 64)
#undef CTREX_NN_UD
    return hipErrorInvalidValue;
}

size_t upconv2_wgrad_scratch(int cin, int cout, long long nvox) {
    const long long chunks = (nvox + wgrad_chunk(nvox) - 1) / wgrad_chunk(nvox);
    return sizeof(float) * static_cast<size_t>(chunks) * 8 * cin * cout;
}

hipError_t launch_upconv2_wgrad(const void *in, int in_cs, int in_off, int cin, const void *dout,
                                int dout_cs, int dout_off, int cout, int D, int H, int W,
                                float *dw, float *scratch, hipStream_t s) {
    const long long nvox = static_cast<long long>(D) * H * W;
    const long long chunk = wgrad_chunk(nvox);
    const int chunks = static_cast<int>((nvox + chunk - 1) / chunk);
    const u16 *ip = static_cast<const u16 *>(in), *dp = static_cast<const u16 *>(dout);
    bool done = false;
#define CTREX_NN_UW(CI, CO)                                                                           \
    if (!done && cin == CI && cout == CO) {                                                            \
        hipLaunchKernelGGL((upconv2_wgrad_kernel<CI, CO>), dim3(chunks, 2), dim3(NT), 0, s, ip, in_cs, \
                           in_off, dp, dout_cs, dout_off, D, H, W, chunk, scratch);                    \
        done = true;                                                                                   \
    }
    CTREX_NN_UW(64, 32)
    CTREX_NN_UW(32, 16)
    CTREX_NN_UW(32, 32)
    CTREX_NN_UW(64, 64)
#undef CTREX_NN_UW
    if (!done) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_wgrad(scratch, chunks, 8, cout, cin, 0, 0, cout, cin, 1, dw, s);
}

hipError_t launch_maxpool2(const void *in, int in_cs, int in_off, int c, void *out, int D, int H,
                           int W, hipStream_t s) {
    const long long n = static_cast<long long>(D / 2) * (H / 2) * (W / 2) * c;
    if (c % 8 == 0 && in_cs % 8 == 0 && in_off % 8 == 0 &&
        (reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) % 16 == 0) {
        hipLaunchKernelGGL(maxpool2_vec8_kernel, dim3(blocks_for(n / 8)), dim3(NT), 0, s,
                           static_cast<const u16 *>(in), in_cs, in_off, c / 8,
                           static_cast<u16 *>(out), D, H, W);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(maxpool2_kernel, dim3(blocks_for(n)), dim3(NT), 0, s,
                       static_cast<const u16 *>(in), in_cs, in_off, c, static_cast<u16 *>(out), D, H, W);
    return hipGetLastError();
}

hipError_t launch_maxpool2_bwd(const void *in, int in_cs, int in_off, int c, const void *dout,
                               void *din, int D, int H, int W, bool relu, hipStream_t s) {
    const long long n = static_cast<long long>(D / 2) * (H / 2) * (W / 2) * c;
    if (relu)
        hipLaunchKernelGGL(maxpool2_bwd_kernel<true>, dim3(blocks_for(n)), dim3(NT), 0, s,
                           static_cast<const u16 *>(in), in_cs, in_off, c,
                           static_cast<const u16 *>(dout), static_cast<u16 *>(din), D, H, W);
    else
        hipLaunchKernelGGL(maxpool2_bwd_kernel<false>, dim3(blocks_for(n)), dim3(NT), 0, s,
                           static_cast<const u16 *>(in), in_cs, in_off, c,
                           static_cast<const u16 *>(dout), static_cast<u16 *>(din), D, H, W);
    return hipGetLastError();
}

hipError_t launch_relu_bwd(const void *y, void *g, int cs, int off, int c, long long nvox,
                           hipStream_t s) {
    const bool vec = cs % 8 == 0 && off % 8 == 0 && c % 8 == 0 &&
                     (reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(g)) % 16 == 0;
    if (vec) {
        const long long n8 = nvox * (c / 8);
        hipLaunchKernelGGL(relu_bwd8_kernel, dim3(blocks_for(n8)), dim3(NT), 0, s,
                           static_cast<const u16 *>(y), static_cast<u16 *>(g), cs, off, c / 8, n8);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks_for(nvox * c)), dim3(NT), 0, s,
                       static_cast<const u16 *>(y), static_cast<u16 *>(g), cs, off, c, nvox);
    return hipGetLastError();
}

hipError_t launch_head(const void *act, int c, const float *h, const float *b, const float *x,
                       float scale, const float *mask, float *out, long long n, hipStream_t s) {
    if (c == 16 && reinterpret_cast<uintptr_t>(act) % 16 == 0)
        hipLaunchKernelGGL((head_vec_kernel<16>), dim3(blocks_for(n)), dim3(NT), 0, s,
                           static_cast<const u16 *>(act), h, b, x, scale, mask, out, n);
    else
        hipLaunchKernelGGL(head_kernel, dim3(blocks_for(n)), dim3(NT), 0, s,
                           static_cast<const u16 *>(act), c, h, b, x, scale, mask, out, n);
    return hipGetLastError();
}

hipError_t launch_scale_bf16(const float *x, float scale, void *xb, long long n, hipStream_t s) {
    hipLaunchKernelGGL(scale_bf16_kernel, dim3(blocks_for(n)), dim3(NT), 0, s, x, scale,
                       static_cast<u16 *>(xb), n);
    return hipGetLastError();
}

constexpr int kHeadBwdBlocks = 2048;

size_t head_bwd_scratch(int c) {
    return sizeof(double) * kHeadBwdBlocks * static_cast<size_t>(c + 1);
}

hipError_t launch_head_bwd(const void *act, int c, const float *h, float scale, const float *mask,
                           const float *dout, void *dact, float *dh, float *db, long long n,
                           bool relu, double *scratch, hipStream_t s) {
    const int blocks = kHeadBwdBlocks;
    if (c != 16) return hipErrorInvalidValue;
    const bool vec = (reinterpret_cast<uintptr_t>(act) | reinterpret_cast<uintptr_t>(dact)) % 16 == 0;
#define CTREX_NN_HB(V, R)                                                                          \
    hipLaunchKernelGGL((head_bwd_kernel<16, V, R>), dim3(blocks), dim3(NT), 0, s,                  \
                       static_cast<const u16 *>(act), h, scale, mask, dout,                        \
                       static_cast<u16 *>(dact), n, scratch)
    if (vec) {
        if (relu) CTREX_NN_HB(true, true);
        else CTREX_NN_HB(true, false);
    } else {
        if (relu) CTREX_NN_HB(false, true);
        else CTREX_NN_HB(false, false);
    }
#undef CTREX_NN_HB
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dh)
        hipLaunchKernelGGL(reduce_rows_kernel, dim3(blocks_for(c, 32)), dim3(RR_THREADS), 0, s,
                           scratch, blocks, c, c + 1, dh);
    if (db)
        hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(RR_THREADS), 0, s, scratch + c,
                           blocks, 1, c + 1, db);
    return hipGetLastError();
}

hipError_t launch_mse(const float *a, const float *t, long long n, float weight, float *grad,
                      double *partial, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3(blocks), dim3(NT), 0, s, a, t, n,
                       static_cast<float>(2.0 * weight / static_cast<double>(n)), grad, partial);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, static_cast<float>(step));
    const float c2 = 1.0f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(NT), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack(const float *w, int cout, int cin, int taps, bool mirror, void *wt,
                       void *wt_d, bool in_major, hipStream_t s) {
    const int n = cout * cin * taps;
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(n)), dim3(NT), 0, s, w, cout, cin, taps,
                       mirror ? 1 : 0, static_cast<u16 *>(wt), static_cast<u16 *>(wt_d), in_major ? 1 : 0);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace ctrex
