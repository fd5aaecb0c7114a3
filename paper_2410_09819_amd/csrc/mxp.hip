// Mixed-precision panel update and tile finalization (Section IV-C).
//
// Each off-diagonal tile has a class (FP64, FP32, FP16, BF16 or FP8 e4m3)
// that decides how it is stored and how the updates into it are computed:
//   C_mk = A_mk - sum_{n<k} Q_p(Lh_mn) Q_p(Lh_kn)^T,   p = class(m, k)
// where Lh are the stored factor tiles and Q_p rounds a stored tile to class
// p with its per-tile scale. Diagonal tiles and FP64-class tiles use FP64
// MFMA on the stored operands, upcast exactly while they are staged into LDS.
// The low classes read "operand copies": for every tile and every low class
// it will be multiplied in (known from the static schedule), the finalize
// step writes Q_p(Lh) in the MFMA operand order (row-major, k contiguous)
// with a power-of-two copy scale. FP16, BF16 and FP8 run on the narrow
// MFMAs with FP32 accumulation. FP32 runs on the FP16 MFMA: each binary32
// operand x (times its copy scale) is held as hi + lo, hi = fp16(x),
// lo = fp16(x - hi), and each product as hi_a hi_b + hi_a lo_b + lo_a hi_b
// (the two-term split of Ootomo and Yokota, 2022). For entries within 2^18
// of the copy's largest, the representation and the dropped lo_a lo_b cost
// at most 3 * 2^-22 of |ab| per product; smaller entries (FP16 subnormal
// lo) are held to 2^-25 absolute in the scaled domain, 2^-40 of the
// largest. Norm-wise this stays below the FP32 accumulation error of the
// K >= 1024 terms a column sums over.
// POTRF and TRSM run in FP64 on a working copy of the column; finalize
// rounds each new tile to its class (with its scale) into the factor
// storage and writes its operand copies.
#include "formats.hpp"
#include "gemm_f64.hpp"

namespace tc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kB = 128;       // output block
constexpr int kStrips = 16;   // strips per tile for amax / cast
constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// FP64 main loop over operands stored in any class (upcast while staging).
//
// A stage is a 128 x 16 operand slab (16 columns of the tile, 128 rows),
// loaded with consecutive lanes on consecutive bytes: a binary64 slab as
// four 16-byte pieces per thread (2 rows each), the other classes as two
// pieces of 4 consecutive rows (16, 8, 8 or 4 bytes each). The raw bits
// stay in registers while the current stage's MFMAs run; after them they
// are decoded to binary64 and written to LDS. An operand's class changes
// only between tile columns, so each tile column's stages run in a loop
// specialized for its (A class, B class) pair: straight-line loads,
// decodes and waits, as in the all-binary64 main loop.
//
// The workgroup is that of the all-binary64 kernels: 256 threads, 2 x 2
// waves of 64 x 64 of the 128 x 128 block, two workgroups per CU, so one
// workgroup's barriers and decodes overlap the other's MFMAs. With 64 x 64
// accumulators per wave, the 25 pair loops inlined into one kernel do not
// fit in 256 registers (the compiler keeps them apart), so each pair loop
// is a function of its own: it takes the accumulators from memory (private
// to the lane) at the start of its tile column and puts them back at the
// end, 64 moves per tile column of 64 stages.
//
// The scaled classes' (FP16, FP8) tile scales are not applied to each
// decoded element: a pair loop runs in a frame of 2^s, s = the sum of its
// operands' scales (the accumulators are divided by 2^s on entry and
// multiplied back on exit). Power-of-two scaling commutes with binary64
// rounding away from the subnormal range, so the sums are those of scaled
// operands, with a third fewer decode instructions.
// ---------------------------------------------------------------------------
struct MixedTile {
    const char* base;  // tile start
    int cls;
    int scale;
};

struct RawSlab {
    uint4 w[4];
};

constexpr int kF64Threads = 256;
constexpr int kF64MI = 4, kF64NI = 4;  // 16 x 16 MFMA blocks per wave

// A thread's pieces of a slab: element offsets in the tile (leading
// dimension nb) and LDS offsets of its first binary64 piece of 2 rows
// (e2, s2; piece q is kQ2 q columns further) or its first piece of 4 rows
// of the narrower classes (e4, s4; the second is kQ4 columns further).
struct SlabMap {
    int e2, s2, e4, s4;
};
constexpr int kQ2 = 2 * kF64Threads / 128;  // columns between binary64 pieces
constexpr int kQ4 = 4 * kF64Threads / 128;  // ... between narrower pieces

template <int LD>
__device__ __forceinline__ SlabMap slab_map(int tid, int nb) {
    SlabMap m;
    const int e2 = tid * 2, e4 = tid * 4;
    m.e2 = (e2 >> 7) * nb + (e2 & 127);
    m.s2 = (e2 >> 7) * LD + (e2 & 127);
    m.e4 = (e4 >> 7) * nb + (e4 & 127);
    m.s4 = (e4 >> 7) * LD + (e4 & 127);
    return m;
}

// Loads through global-address-space pointers: the pair loops are
// functions, where a plain pointer would make flat loads (which the LDS
// waits would then also wait for).
#define TC_GLOBAL __attribute__((address_space(1)))
typedef unsigned gu4v __attribute__((ext_vector_type(4)));
typedef unsigned gu2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint4 to_u4(gu4v v) { return uint4{v.x, v.y, v.z, v.w}; }

// Raw bits of a thread's pieces of the class-C slab starting at element idx.
template <int C>
__device__ __forceinline__ void raw_load(const char* base, int64_t idx, int64_t nb,
                                         const SlabMap& m, RawSlab& r) {
    const TC_GLOBAL char* g = (const TC_GLOBAL char*)base;
    if constexpr (C == kFP64) {
        const TC_GLOBAL double* p = (const TC_GLOBAL double*)g + idx + m.e2;
#pragma unroll
        for (int q = 0; q < 4; ++q) r.w[q] = to_u4(*(const TC_GLOBAL gu4v*)(p + q * kQ2 * nb));
    } else if constexpr (C == kFP32) {
        const TC_GLOBAL float* p = (const TC_GLOBAL float*)g + idx + m.e4;
#pragma unroll
        for (int q = 0; q < 2; ++q) r.w[q] = to_u4(*(const TC_GLOBAL gu4v*)(p + q * kQ4 * nb));
    } else if constexpr (C == kFP16 || C == kBF16) {
        const TC_GLOBAL uint16_t* p = (const TC_GLOBAL uint16_t*)g + idx + m.e4;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const gu2v v = *(const TC_GLOBAL gu2v*)(p + q * kQ4 * nb);
            r.w[q].x = v.x;
            r.w[q].y = v.y;
        }
    } else {
        const TC_GLOBAL uint8_t* p = (const TC_GLOBAL uint8_t*)g + idx + m.e4;
#pragma unroll
        for (int q = 0; q < 2; ++q) r.w[q].x = *(const TC_GLOBAL uint32_t*)(p + q * kQ4 * nb);
    }
}

typedef float f2v __attribute__((ext_vector_type(2)));

// A 4-row piece of a narrower class in binary64, unscaled. Conversions are
// exact: FP8 (OCP e4m3, which the gfx950 packed conversion implements) and
// FP16 through binary32.
template <int C>
__device__ __forceinline__ void decode_piece(const uint4 w, double (&v)[4]) {
    if constexpr (C == kFP32) {
        v[0] = (double)__uint_as_float(w.x);
        v[1] = (double)__uint_as_float(w.y);
        v[2] = (double)__uint_as_float(w.z);
        v[3] = (double)__uint_as_float(w.w);
    } else if constexpr (C == kFP16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t h = ((i < 2 ? w.x : w.y) >> (16 * (i & 1))) & 0xFFFFu;
            v[i] = (double)(float)__builtin_bit_cast(_Float16, (uint16_t)h);
        }
    } else if constexpr (C == kBF16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t h = ((i < 2 ? w.x : w.y) >> (16 * (i & 1))) & 0xFFFFu;
            v[i] = (double)__uint_as_float(h << 16);
        }
    } else {
        const f2v lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w.x, false);
        const f2v hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w.x, true);
        v[0] = lo.x;
        v[1] = lo.y;
        v[2] = hi.x;
        v[3] = hi.y;
    }
}

// Decode a thread's pieces of a class-C slab and write them to the LDS
// stage dst.
template <int C, int LD>
__device__ __forceinline__ void raw_store(const RawSlab& r, const SlabMap& m, double* dst) {
    if constexpr (C == kFP64) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 w = r.w[q];
            *reinterpret_cast<d2*>(dst + m.s2 + q * kQ2 * LD) =
                d2{__hiloint2double((int)w.y, (int)w.x), __hiloint2double((int)w.w, (int)w.z)};
        }
    } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            double v[4];
            decode_piece<C>(r.w[q], v);
            *reinterpret_cast<d2*>(dst + m.s4 + q * kQ4 * LD) = d2{v[0], v[1]};
            *reinterpret_cast<d2*>(dst + m.s4 + q * kQ4 * LD + 2) = d2{v[2], v[3]};
        }
    }
}

typedef d4 F64Acc[kF64MI][kF64NI];

// Stages c0, c0 + 16, ... < c1 (columns of tile column n) with A of class CA
// (tile at abase) and B of class CB (at bbase): the double-buffered loop of
// the all-binary64 main loop, its first stage loaded without overlap.
// a0, b0: element offsets of the slabs' first row in column 0 of their
// tiles.
template <int CA, int CB>
__device__ __forceinline__ void mixed_run_body(F64Acc& acc, const char* abase, const char* bbase,
                                               int64_t a0, int64_t b0, int64_t nb, int c0, int c1,
                                               const SlabMap& map, double* lds) {
    using T = MfmaTile<kB, kB>;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    double* As = lds;
    double* Bs = lds + 2 * T::BK * T::LDA;
    RawSlab ra, rb;
    raw_load<CA>(abase, a0 + (int64_t)c0 * nb, nb, map, ra);
    raw_load<CB>(bbase, b0 + (int64_t)c0 * nb, nb, map, rb);
    raw_store<CA, T::LDA>(ra, map, As);
    raw_store<CB, T::LDB>(rb, map, Bs);
    __syncthreads();
    int buf = 0;
    const int li = lane & 15, lk = lane >> 4;
    for (int c = c0; c < c1; c += T::BK) {
        const bool more = c + T::BK < c1;
        if (more) {
            raw_load<CA>(abase, a0 + (int64_t)(c + T::BK) * nb, nb, map, ra);
            raw_load<CB>(bbase, b0 + (int64_t)(c + T::BK) * nb, nb, map, rb);
        }
        const double* as = As + buf * T::BK * T::LDA + wm * 64 + li;
        const double* bs = Bs + buf * T::BK * T::LDB + wn * 64 + li;
#pragma unroll
        for (int ks = 0; ks < T::BK / 4; ++ks) {
            const int k = ks * 4 + lk;
            double a[kF64MI], b[kF64NI];
#pragma unroll
            for (int mi = 0; mi < kF64MI; ++mi) a[mi] = as[k * T::LDA + mi * 16];
#pragma unroll
            for (int ni = 0; ni < kF64NI; ++ni) b[ni] = bs[k * T::LDB + ni * 16];
#pragma unroll
            for (int mi = 0; mi < kF64MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < kF64NI; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[ni], a[mi], acc[mi][ni],
                                                                      0, 0, 0);
        }
        if (more) {
            raw_store<CA, T::LDA>(ra, map, As + (buf ^ 1) * T::BK * T::LDA);
            raw_store<CB, T::LDB>(rb, map, Bs + (buf ^ 1) * T::BK * T::LDB);
        }
        __syncthreads();
        buf ^= 1;
    }
}

// Wave-uniform copy of a 64-bit value: a function's arguments arrive in
// vector registers, and loop control and address bases belong in scalar
// ones.
__device__ __forceinline__ int64_t uni64(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The pair loop of one tile column, a function of its own: the
// accumulators come in from accm (lane-private memory) divided by 2^s, the
// frame of the operands' scales, and go back multiplied by it.
template <int CA, int CB>
__device__ __attribute__((noinline)) void mixed_run(F64Acc& accm, const MixedTile ta,
                                                    const MixedTile tb, int64_t a0, int64_t b0,
                                                    int64_t nb, int c0, int c1, const SlabMap map,
                                                    double* lds) {
    const int s = __builtin_amdgcn_readfirstlane((CA == kFP16 || CA == kFP8 ? ta.scale : 0) +
                                                 (CB == kFP16 || CB == kFP8 ? tb.scale : 0));
    F64Acc acc;
#pragma unroll
    for (int mi = 0; mi < kF64MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < kF64NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[mi][ni][v] = ldexp(accm[mi][ni][v], -s);
    mixed_run_body<CA, CB>(acc, (const char*)uni64((int64_t)ta.base),
                           (const char*)uni64((int64_t)tb.base), uni64(a0), uni64(b0), uni64(nb),
                           __builtin_amdgcn_readfirstlane(c0), __builtin_amdgcn_readfirstlane(c1),
                           map, (double*)uni64((int64_t)lds));
#pragma unroll
    for (int mi = 0; mi < kF64MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < kF64NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) accm[mi][ni][v] = ldexp(acc[mi][ni][v], s);
}

template <int CA>
__device__ __forceinline__ void mixed_run_b(F64Acc& acc, const MixedTile& ta, const MixedTile& tb,
                                            int64_t a0, int64_t b0, int64_t nb, int c0, int c1,
                                            const SlabMap& map, double* lds) {
    switch (tb.cls) {
        case kFP64: mixed_run<CA, kFP64>(acc, ta, tb, a0, b0, nb, c0, c1, map, lds); break;
        case kFP32: mixed_run<CA, kFP32>(acc, ta, tb, a0, b0, nb, c0, c1, map, lds); break;
        case kFP16: mixed_run<CA, kFP16>(acc, ta, tb, a0, b0, nb, c0, c1, map, lds); break;
        case kBF16: mixed_run<CA, kBF16>(acc, ta, tb, a0, b0, nb, c0, c1, map, lds); break;
        default: mixed_run<CA, kFP8>(acc, ta, tb, a0, b0, nb, c0, c1, map, lds); break;
    }
}

// acc += A B^T over the K range [kbeg, kend) (a multiple of 16 long, kbeg
// a multiple of 16): tile column by tile column, each in the loop of its
// classes.
template <class AOp, class BOp>
__device__ __forceinline__ void mixed_mainloop(F64Acc& acc, const AOp& aop, const BOp& bop,
                                               int64_t nb, int64_t kbeg, int64_t kend, double* lds) {
    using T = MfmaTile<kB, kB>;
    static_assert(kB * T::BK == 8 * kF64Threads, "eight slab elements per thread per operand");
    static_assert(T::LDA == T::LDB, "one slab map for both operands");
    const SlabMap map = slab_map<T::LDA>(threadIdx.x, (int)nb);
    for (int64_t kk = kbeg; kk < kend;) {
        const int64_t n = kk / nb;
        const int c0 = (int)(kk - n * nb);
        const int c1 = (int)((kend - n * nb) < nb ? (kend - n * nb) : nb);
        const MixedTile ta = aop.tile(n), tb = bop.tile(n);
        switch (ta.cls) {
            case kFP64: mixed_run_b<kFP64>(acc, ta, tb, aop.r0, bop.r0, nb, c0, c1, map, lds); break;
            case kFP32: mixed_run_b<kFP32>(acc, ta, tb, aop.r0, bop.r0, nb, c0, c1, map, lds); break;
            case kFP16: mixed_run_b<kFP16>(acc, ta, tb, aop.r0, bop.r0, nb, c0, c1, map, lds); break;
            case kBF16: mixed_run_b<kBF16>(acc, ta, tb, aop.r0, bop.r0, nb, c0, c1, map, lds); break;
            default: mixed_run_b<kFP8>(acc, ta, tb, aop.r0, bop.r0, nb, c0, c1, map, lds); break;
        }
        kk += c1 - c0;
    }
}

// Stored tiles (row_tile, n) of the factor as MixedTiles; r0 = the slab's
// first row inside the tile.
struct StoredOp {
    const char* storage;
    const int64_t* toff;
    const uint8_t* tcls;
    const int* tscl;
    int64_t Nt, nb, row_tile, r0;
    __device__ MixedTile tile(int64_t n) const {
        const int64_t t = tile_off(Nt, row_tile, n);
        return MixedTile{storage + toff[t], (int)tcls[t], tscl[t]};
    }
};

// Decode logical block b of a class group: the diagonal tile's lower
// blocks first (when the group includes it), then T x T blocks per listed
// row tile.
__device__ __forceinline__ void group_block(int64_t b, int T, bool diag, const int* rows,
                                            int64_t& rt, int& br, int& bc) {
    const int64_t tri = diag ? (int64_t)T * (T + 1) / 2 : 0;
    if (b < tri) {
        int r = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((int64_t)(r + 1) * (r + 2) / 2 <= b) ++r;
        while ((int64_t)r * (r + 1) / 2 > b) --r;
        rt = 0;
        br = r;
        bc = (int)(b - (int64_t)r * (r + 1) / 2);
    } else {
        const int64_t b2 = b - tri;
        rt = rows[b2 / ((int64_t)T * T)];
        const int w = (int)(b2 % ((int64_t)T * T));
        br = w / T;
        bc = w % T;
    }
}

// FP64 group of column k: W[rt] -= sum_n Lh(k+rt, n) Lh(k, n)^T over the K
// range [K0, K1) (tile columns n of the range), for rt in the diagonal tile
// (lower blocks, when diag) and the listed row tiles. splits > 1: split s
// covers [K0 + s*kchunk, K0 + (s+1)*kchunk) and writes its 128 x 128 block
// to partial[(s * nblocks + b) * 128^2] (column-major).
__global__ __launch_bounds__(kF64Threads, 2) void mxp_gemm_f64_kernel(
    double* __restrict__ W, int Nt, int nb, int k, int64_t K0, int64_t K1,
    const int* __restrict__ rows, int nrows, int diag, const char* __restrict__ storage,
    const int64_t* __restrict__ toff, const uint8_t* __restrict__ tcls,
    const int* __restrict__ tscl, int splits, int64_t kchunk, double* __restrict__ partial) {
    using Tl = MfmaTile<kB, kB>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int T = nb / kB;
    const int64_t nblocks = (diag ? (int64_t)T * (T + 1) / 2 : 0) + (int64_t)nrows * T * T;
    const int64_t logical = xcd_remap(blockIdx.x, nblocks * splits);
    const int split = (int)(logical / nblocks);
    const int64_t b = logical - (int64_t)split * nblocks;
    int64_t rt;
    int br, bc;
    group_block(b, T, diag != 0, rows, rt, br, bc);
    const int64_t kbeg = K0 + (int64_t)split * kchunk;
    const int64_t kend = kbeg + kchunk < K1 ? kbeg + kchunk : K1;
    F64Acc acc;
#pragma unroll
    for (int mi = 0; mi < kF64MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < kF64NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const StoredOp aop{storage, toff, tcls, tscl, Nt, nb, k + rt, (int64_t)br * kB};
    const StoredOp bop{storage, toff, tcls, tscl, Nt, nb, k, (int64_t)bc * kB};
    mixed_mainloop(acc, aop, bop, nb, kbeg, kend, lds);
    double* out;
    int64_t ldo;
    if (splits == 1) {
        out = W + rt * (int64_t)nb * nb + (int64_t)bc * kB * nb + br * kB;
        ldo = nb;
    } else {
        out = partial + ((int64_t)split * nblocks + b) * kB * kB;
        ldo = kB;
    }
    // element v of block (mi, ni): row 64 wm + 16 mi + l % 16, column
    // 32 wn + 16 ni + l / 16 + 4 v (the transposed-block layout of the
    // binary64 kernels)
#pragma unroll
    for (int mi = 0; mi < kF64MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < kF64NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double* p = out + (int64_t)acc_col<kB, kB>(ni, v) * ldo + acc_row<kB, kB>(mi);
                if (splits == 1)
                    *p -= acc[mi][ni][v];
                else
                    *p = acc[mi][ni][v];
            }
}

// W block -= sum over splits of its partial blocks (fixed order).
__global__ __launch_bounds__(256) void mxp_group_reduce_kernel(double* __restrict__ W, int nb,
                                                               const int* __restrict__ rows,
                                                               int diag, int64_t nblocks,
                                                               int splits,
                                                               const double* __restrict__ partial) {
    const int64_t b = blockIdx.x;
    const int T = nb / kB;
    int64_t rt;
    int br, bc;
    group_block(b, T, diag != 0, rows, rt, br, bc);
    double* out = W + rt * (int64_t)nb * nb + (int64_t)bc * kB * nb + br * kB;
    for (int e = threadIdx.x * 2; e < kB * kB; e += 512) {
        const int c = e / kB, r = e - c * kB;
        d2 s = *reinterpret_cast<const d2*>(partial + b * kB * kB + e);
        for (int sp = 1; sp < splits; ++sp)
            s += *reinterpret_cast<const d2*>(partial + ((int64_t)sp * nblocks + b) * kB * kB + e);
        d2* o = reinterpret_cast<d2*>(out + (int64_t)c * nb + r);
        *o = *o - s;
    }
}

// ---------------------------------------------------------------------------
// Finalize the tiles below the diagonal of column k: amax, then rounding to
// the tile's class with its scale, and the operand copies.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void tile_amax_kernel(const double* __restrict__ W, int nb,
                                                             double* __restrict__ part) {
    __shared__ double red[kThreads / 64];
    const int rt = blockIdx.y, strip = blockIdx.x;
    const int64_t per = (int64_t)nb * nb / kStrips;
    const double* p = W + (int64_t)rt * nb * nb + strip * per;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < per; i += kThreads) m = fmax(m, fabs(p[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < kThreads / 64; ++w) t = fmax(t, red[w]);
        part[rt * kStrips + strip] = t;
    }
}

// One workgroup per 64 x 64 block of a new tile: round to the tile's
// class with its scale into storage (column-major), then write the operand
// copies with the copy's own scale, transposed through LDS so each copy is
// row-major (64 consecutive k per row and block): the class's bits for
// FP16 / BF16 / FP8, and for FP32 the binary32 value split into an FP16 hi
// plane and an FP16 lo plane (the lo plane nb * nb halves after the hi
// plane; the scale is chosen for FP16's range).
constexpr int kCB = 64;
constexpr int kCPitch = kCB * 2 + 16;  // bytes per staged copy row

// Rounding of one 64 x 64 block into the operand copies (LDS staging, then
// row-major writes). v(i) gives the stored factor value of element i.
template <class V>
__device__ __forceinline__ void write_copies(const V& val, int nb, int r0, int c0, char* const* copy,
                                             const int* ce, uint8_t (*stage)[kCB * kCPitch]) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int j = 0; j < kCB / 4; ++j) {
        const int cl = ty + 4 * j;
        const int64_t i = (int64_t)(c0 + cl) * nb + r0 + tx;
        const double v = val(i);
        if (copy[kFP32]) {
            // x - hi is exact in binary64; hi and lo saturate like any FP16 value
            const double x = ldexp(round_to_class(v, kFP32), -ce[kFP32]);
            const double hi = round_to_class(x, kFP16);
            *reinterpret_cast<uint16_t*>(&stage[3][tx * kCPitch + 2 * cl]) = enc_fp16(hi);
            *reinterpret_cast<uint16_t*>(&stage[4][tx * kCPitch + 2 * cl]) =
                enc_fp16(round_to_class(x - hi, kFP16));
        }
        if (copy[kFP16]) {
            const uint16_t b = enc_fp16(round_to_class(ldexp(v, -ce[kFP16]), kFP16));
            *reinterpret_cast<uint16_t*>(&stage[0][tx * kCPitch + 2 * cl]) = b;
        }
        if (copy[kBF16]) {
            const uint16_t b = enc_bf16(round_to_class(ldexp(v, -ce[kBF16]), kBF16));
            *reinterpret_cast<uint16_t*>(&stage[1][tx * kCPitch + 2 * cl]) = b;
        }
        if (copy[kFP8])
            stage[2][tx * kCPitch + cl] = enc_fp8(round_to_class(ldexp(v, -ce[kFP8]), kFP8));
    }
    __syncthreads();
    // row-major copies: row r0 + rr holds k = c0 .. c0 + 63 contiguously
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int c2 = q < 3 ? kFP16 + q : kFP32;
        if (!copy[c2]) continue;
        const int eb = q < 3 ? fmt_bytes(c2) : 2;
        char* dc = copy[c2] + (q == 4 ? (int64_t)nb * nb * 2 : 0);
        const int per_row = kCB * eb / 16;  // 16-byte chunks per row
        for (int ch = threadIdx.x; ch < kCB * per_row; ch += kThreads) {
            const int rr = ch / per_row, cc = ch - rr * per_row;
            const uint4 v = *reinterpret_cast<const uint4*>(&stage[q][rr * kCPitch + cc * 16]);
            *reinterpret_cast<uint4*>(dc + ((int64_t)(r0 + rr) * nb + c0) * eb + cc * 16) = v;
        }
    }
}

__global__ __launch_bounds__(kThreads) void tile_cast_kernel(
    const double* __restrict__ W, int Nt, int nb, int k, const double* __restrict__ part,
    char* __restrict__ storage, const int64_t* __restrict__ toff, const uint8_t* __restrict__ tcls,
    int* __restrict__ tscl, const int64_t* __restrict__ shoff, int* __restrict__ cscl) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[5][kCB * kCPitch];
    const int rt = blockIdx.z;  // tile k + 1 + rt of column k
    const int r0 = blockIdx.x * kCB, c0 = blockIdx.y * kCB;
    const int64_t t = tile_off(Nt, k + 1 + rt, k);
    double amax = 0.0;
    for (int s = 0; s < kStrips; ++s) amax = fmax(amax, part[rt * kStrips + s]);
    const int c = tcls[t];
    const int e = class_scale(amax, c);
    // largest stored value (rounding is monotone): decides the copies' scales
    const double amax_h = ldexp(fabs(round_to_class(ldexp(amax, -e), c)), e);
    int ce[5];
    char* copy[5];
#pragma unroll
    for (int c2 = 1; c2 <= 4; ++c2) {
        const int64_t o = shoff[t * 4 + (c2 - 1)];
        copy[c2] = o >= 0 ? storage + o : nullptr;
        ce[c2] = class_scale(amax_h, c2 == kFP32 ? kFP16 : c2);
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        tscl[t] = e;
        for (int c2 = 1; c2 <= 4; ++c2) cscl[t * 4 + (c2 - 1)] = ce[c2];
    }
    const double* src = W + (int64_t)(1 + rt) * nb * nb;
    void* dst = storage + toff[t];
    auto val = [=](int64_t i) {
        const double r = round_to_class(ldexp(src[i], -e), c);
        store_elem(dst, i, c, r);
        return ldexp(r, e);  // the stored factor value
    };
    write_copies(val, nb, r0, c0, copy, ce, stage);
}

// Operand copies of stored tiles list[z] (tiles already in storage, their
// scales in tscl / cscl): the same values tile_cast_kernel wrote when the
// tiles were finalized, rebuilt from the stored bits.
__global__ __launch_bounds__(kThreads) void tile_copies_kernel(
    int nb, const int* __restrict__ list, char* __restrict__ storage,
    const int64_t* __restrict__ toff, const uint8_t* __restrict__ tcls,
    const int* __restrict__ tscl, const int64_t* __restrict__ shoff,
    const int* __restrict__ cscl) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[5][kCB * kCPitch];
    const int64_t t = list[blockIdx.z];
    const int r0 = blockIdx.x * kCB, c0 = blockIdx.y * kCB;
    const int c = tcls[t], e = tscl[t];
    int ce[5];
    char* copy[5];
#pragma unroll
    for (int c2 = 1; c2 <= 4; ++c2) {
        const int64_t o = shoff[t * 4 + (c2 - 1)];
        copy[c2] = o >= 0 ? storage + o : nullptr;
        ce[c2] = cscl[t * 4 + (c2 - 1)];
    }
    const void* src = storage + toff[t];
    auto val = [=](int64_t i) { return load_elem(src, i, c, e); };
    write_copies(val, nb, r0, c0, copy, ce, stage);
}

// Tables of an out-of-core mixed factor: upd[2i] = tile t, upd[2i + 1] =
// byte offset of its slot (stored tile first, then the copy areas at
// coff[c - 1] for the copy classes the tile needs: bit c of need[t]).
__global__ void slot_tables_kernel(const int64_t* __restrict__ upd, int count,
                                   const uint8_t* __restrict__ need, int64_t c1, int64_t c2,
                                   int64_t c3, int64_t c4, int64_t* __restrict__ toff,
                                   int64_t* __restrict__ shoff) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t t = upd[2 * i], base = upd[2 * i + 1];
    const int64_t coff[4] = {c1, c2, c3, c4};
    toff[t] = base;
    for (int c = 1; c <= 4; ++c)
        shoff[t * 4 + (c - 1)] = (need[t] >> c) & 1 ? base + coff[c - 1] : -1;
}

// ---------------------------------------------------------------------------
// Narrow-format MFMA for the FP16, BF16 and FP8 groups. Operands are the
// row-major copies: a 128-row slab of 128 bytes per row per stage (64 k of
// FP16/BF16, 128 k of FP8) is staged through LDS in two 64-byte planes;
// lane l of a wave takes row l % 16 and chunk l / 16 of a plane: 8 k per
// plane for the 16-bit formats (one MFMA per plane), and the chunk of both
// planes (32 k) for FP8 -- A and B use the same k order, which is all the
// MFMA needs. v_mfma_f32_16x16x32_{f16,bf16} and
// v_mfma_scale_f32_16x16x128_f8f6f4 (unit scales) accumulate in FP32; lane
// l holds D[4(l/16) + v][l%16] (checked on the device) and the blocks are
// computed as C^T = B A^T. The per-tile copy scales 2^(e_a + e_b) are
// applied (ldexp per element) when the products of one tile column n are
// folded into the FP32 accumulator.
// ---------------------------------------------------------------------------
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));

constexpr int kNPitch = 128 + 16;  // bytes per LDS row (bank spread)

struct NarrowOp {
    const char* storage;
    const int64_t* shoff;
    const int* cscl;
    int cls;
    int64_t Nt, nb, row_tile, r0;
    __device__ const uint8_t* rows(int64_t n, int eb) const {
        const int64_t t = tile_off(Nt, row_tile, n);
        return reinterpret_cast<const uint8_t*>(storage + shoff[t * 4 + (cls - 1)]) + r0 * nb * eb;
    }
    __device__ int scale(int64_t n) const { return cscl[tile_off(Nt, row_tile, n) * 4 + (cls - 1)]; }
};

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// LDS layout of the narrow and split kernels: an operand's stage rows are
// held in planes of 128 rows x 64 bytes (no padding), and 16-byte chunk c of
// row r sits at chunk c ^ ((r >> 1) & 3) of its plane row. Both the MFMA
// operand reads (16 lanes: 16 rows, one chunk) and the stores of the
// coalesced loads (4 lanes per row) are then free of bank conflicts on
// gfx950 (checked with the LDS bank-conflict counter; padded pitches of 80
// or 144 bytes are not, for the reads).
constexpr int kPlane = kB * 64;  // bytes per plane
__device__ __forceinline__ int swz(int r, int c) { return r * 64 + 16 * (c ^ ((r >> 1) & 3)); }

struct Quad {
    u4v v0, v1, v2, v3;
};
// A thread's four 16-byte pieces of a 128-byte stage row: rows r and r + 64
// (step = 64 rows), bytes c and c + 64; in LDS, plane 0 holds bytes 0..63
// of each row and plane 1 bytes 64..127 (p = the swizzled slot of (r, c)).
__device__ __forceinline__ void load_quad(const uint8_t* p, int64_t step, Quad& q) {
    q.v0 = *reinterpret_cast<const u4v*>(p);
    q.v1 = *reinterpret_cast<const u4v*>(p + step);
    q.v2 = *reinterpret_cast<const u4v*>(p + 64);
    q.v3 = *reinterpret_cast<const u4v*>(p + step + 64);
}
__device__ __forceinline__ void store_quad(uint8_t* p, const Quad& q) {
    *reinterpret_cast<u4v*>(p) = q.v0;
    *reinterpret_cast<u4v*>(p + 64 * 64) = q.v1;
    *reinterpret_cast<u4v*>(p + kPlane) = q.v2;
    *reinterpret_cast<u4v*>(p + kPlane + 64 * 64) = q.v3;
}

template <int CLS>
__global__ __launch_bounds__(kGemmThreads, 2) void mxp_gemm_narrow_kernel(
    double* __restrict__ W, int Nt, int nb, int k, int nbeg, int nend, const int* __restrict__ rows,
    int nrows, const char* __restrict__ storage, const int64_t* __restrict__ shoff,
    const int* __restrict__ cscl) {
    constexpr int EB = CLS == kFP8 ? 1 : 2;
    constexpr int SK = 128 / EB;  // k per stage
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][2][2 * kPlane];  // [buf][A, B][plane]
    const int T = nb / kB;
    const int64_t total = (int64_t)nrows * T * T;
    const int64_t b = xcd_remap(blockIdx.x, total);
    int64_t rt;
    int br, bc;
    group_block(b, T, false, rows, rt, br, bc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 15, lg = lane >> 4;
    const NarrowOp aop{storage, shoff, cscl, CLS, Nt, nb, k + rt, (int64_t)br * kB};
    const NarrowOp bop{storage, shoff, cscl, CLS, Nt, nb, k, (int64_t)bc * kB};
    const int spt = nb / SK;  // stages per tile column
    const int g0 = nbeg * spt, g1 = nend * spt;
    // thread t moves rows t / 4 and t / 4 + 64, bytes 16 (t % 4) and 64 more
    // of the 128-byte stage row (4 lanes read 64 contiguous bytes of a row)
    const int lrow = tid >> 2, lch = tid & 3;
    const int64_t gstep = (int64_t)64 * nb * EB;  // 64 rows further
    const int64_t lofs = (int64_t)lrow * nb * EB + 16 * lch;
    const int so = swz(lrow, lch);
    // MFMA operand slot of this lane: row 16 i + l % 16, chunk l / 16
    const int ro = swz(li, lg);
    Quad ra, rb;
    f4 acc[4][4], part[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            acc[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
            part[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
        }
    if (g1 > g0) {
        load_quad(aop.rows(nbeg, EB) + lofs, gstep, ra);
        load_quad(bop.rows(nbeg, EB) + lofs, gstep, rb);
        store_quad(&lds[0][0][so], ra);
        store_quad(&lds[0][1][so], rb);
        __syncthreads();
        int buf = 0;
        for (int g = g0; g < g1; ++g) {
            const bool more = g + 1 < g1;
            if (more) {
                const int n1 = (g + 1) / spt, st1 = (g + 1) - n1 * spt;
                const int64_t o = lofs + (int64_t)st1 * SK * EB;
                load_quad(aop.rows(n1, EB) + o, gstep, ra);
                load_quad(bop.rows(n1, EB) + o, gstep, rb);
            }
            const uint8_t* as = &lds[buf][0][wm * 64 * 64 + ro];
            const uint8_t* bs = &lds[buf][1][wn * 64 * 64 + ro];
            if constexpr (CLS == kFP8) {
                // lane group l / 16 takes chunk l / 16 of both planes (32 k);
                // A and B use the same k order
                i8v a[4], bq[4];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) {
                    const u4v x = *reinterpret_cast<const u4v*>(as + mi * 16 * 64);
                    const u4v y = *reinterpret_cast<const u4v*>(as + kPlane + mi * 16 * 64);
                    a[mi] = i8v{(int)x.x, (int)x.y, (int)x.z, (int)x.w, (int)y.x, (int)y.y, (int)y.z, (int)y.w};
                }
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    const u4v x = *reinterpret_cast<const u4v*>(bs + ni * 16 * 64);
                    const u4v y = *reinterpret_cast<const u4v*>(bs + kPlane + ni * 16 * 64);
                    bq[ni] = i8v{(int)x.x, (int)x.y, (int)x.z, (int)x.w, (int)y.x, (int)y.y, (int)y.z, (int)y.w};
                }
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        part[mi][ni] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                            bq[ni], a[mi], part[mi][ni], 0, 0, 0, 127, 0, 127);
            } else {
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {  // plane ks: k 32 ks .. 32 ks + 31
                    u4v a[4], bq[4];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
                        a[mi] = *reinterpret_cast<const u4v*>(as + ks * kPlane + mi * 16 * 64);
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        bq[ni] = *reinterpret_cast<const u4v*>(bs + ks * kPlane + ni * 16 * 64);
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 4; ++ni) {
                            if constexpr (CLS == kFP16)
                                part[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                    __builtin_bit_cast(h8v, bq[ni]), __builtin_bit_cast(h8v, a[mi]),
                                    part[mi][ni], 0, 0, 0);
                            else
                                part[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    __builtin_bit_cast(b8v, bq[ni]), __builtin_bit_cast(b8v, a[mi]),
                                    part[mi][ni], 0, 0, 0);
                        }
                }
            }
            if ((g + 1) % spt == 0) {  // tile column n done: fold with its scales
                const int n = g / spt;
                const int sc = aop.scale(n) + bop.scale(n);
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[mi][ni][v] += ldexpf(part[mi][ni][v], sc);
                        part[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
            if (more) {
                store_quad(&lds[buf ^ 1][0][so], ra);
                store_quad(&lds[buf ^ 1][1][so], rb);
            }
            __syncthreads();
            buf ^= 1;
        }
    }
    double* out = W + rt * (int64_t)nb * nb + (int64_t)bc * kB * nb + br * kB;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * (kB / 2) + mi * 16 + li;
                const int col = wn * (kB / 2) + ni * 16 + 4 * lg + v;
                out[(int64_t)col * nb + row] -= (double)acc[mi][ni][v];
            }
}

// ---------------------------------------------------------------------------
// FP32 group on the FP16 MFMA, with the two-term split of each operand
// (described at the top of this file). Per stage, 32 k of each of the four
// copies (A hi, A lo, B hi, B lo) are staged through LDS as one swizzled
// plane each; lane l takes row l % 16 and k = 8 (l / 16) .. 8 (l / 16) + 7.
// Three v_mfma_f32_16x16x32_f16 per 16 x 16 block and stage; the products of
// one tile column n are folded into the accumulator with the copies' scales
// 2^(e_a + e_b) (ldexp per element, so no scale underflows on its own).
// ---------------------------------------------------------------------------
constexpr int kSK = 32;  // k per stage

struct Pair {
    u4v v0, v1;
};
__device__ __forceinline__ void load_pair(const uint8_t* p, int64_t step, Pair& q) {
    q.v0 = *reinterpret_cast<const u4v*>(p);
    q.v1 = *reinterpret_cast<const u4v*>(p + step);
}
__device__ __forceinline__ void store_pair(uint8_t* p, const Pair& q) {
    *reinterpret_cast<u4v*>(p) = q.v0;
    *reinterpret_cast<u4v*>(p + 64 * 64) = q.v1;  // row + 64: same swizzle
}

__global__ __launch_bounds__(kGemmThreads, 2) void mxp_gemm_split_kernel(
    double* __restrict__ W, int Nt, int nb, int k, int nbeg, int nend, const int* __restrict__ rows,
    int nrows, const char* __restrict__ storage, const int64_t* __restrict__ shoff,
    const int* __restrict__ cscl) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][4][kPlane];
    const int T = nb / kB;
    const int64_t total = (int64_t)nrows * T * T;
    const int64_t b = xcd_remap(blockIdx.x, total);
    int64_t rt;
    int br, bc;
    group_block(b, T, false, rows, rt, br, bc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 15, lg = lane >> 4;
    const NarrowOp aop{storage, shoff, cscl, kFP32, Nt, nb, k + rt, (int64_t)br * kB};
    const NarrowOp bop{storage, shoff, cscl, kFP32, Nt, nb, k, (int64_t)bc * kB};
    const int spt = nb / kSK;  // stages per tile column
    const int g0 = nbeg * spt, g1 = nend * spt;
    // thread t moves rows t / 4 and t / 4 + 64, bytes 16 (t % 4) of the
    // 64-byte stage row of each copy
    const int lrow = tid >> 2, lch = tid & 3;
    const int64_t gstep = (int64_t)64 * nb * 2;
    const int64_t lofs = (int64_t)lrow * nb * 2 + 16 * lch;
    const int64_t plane = (int64_t)nb * nb * 2;  // lo copy after the hi copy
    const int so = swz(lrow, lch);
    const int ro = swz(li, lg);  // MFMA operand slot: row 16 i + l % 16, chunk l / 16
    Pair rah, ral, rbh, rbl;
    f4 acc[4][4], part[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            acc[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
            part[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
        }
    if (g1 > g0) {
        {
            const uint8_t* pa = aop.rows(nbeg, 2) + lofs;
            const uint8_t* pb = bop.rows(nbeg, 2) + lofs;
            load_pair(pa, gstep, rah);
            load_pair(pa + plane, gstep, ral);
            load_pair(pb, gstep, rbh);
            load_pair(pb + plane, gstep, rbl);
        }
        store_pair(&lds[0][0][so], rah);
        store_pair(&lds[0][1][so], ral);
        store_pair(&lds[0][2][so], rbh);
        store_pair(&lds[0][3][so], rbl);
        __syncthreads();
        int buf = 0;
        for (int g = g0; g < g1; ++g) {
            const bool more = g + 1 < g1;
            if (more) {
                const int n1 = (g + 1) / spt, st1 = (g + 1) - n1 * spt;
                const int64_t o = lofs + (int64_t)st1 * kSK * 2;
                const uint8_t* pa = aop.rows(n1, 2) + o;
                const uint8_t* pb = bop.rows(n1, 2) + o;
                load_pair(pa, gstep, rah);
                load_pair(pa + plane, gstep, ral);
                load_pair(pb, gstep, rbh);
                load_pair(pb + plane, gstep, rbl);
            }
            const int ao = wm * 64 * 64 + ro;
            const int bo = wn * 64 * 64 + ro;
            u4v xa[4], xb[4], ya[4];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
                xa[mi] = *reinterpret_cast<const u4v*>(&lds[buf][0][ao + mi * 16 * 64]);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                xb[ni] = *reinterpret_cast<const u4v*>(&lds[buf][2][bo + ni * 16 * 64]);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    part[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(h8v, xb[ni]), __builtin_bit_cast(h8v, xa[mi]),
                        part[mi][ni], 0, 0, 0);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
                ya[mi] = *reinterpret_cast<const u4v*>(&lds[buf][1][ao + mi * 16 * 64]);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    part[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(h8v, xb[ni]), __builtin_bit_cast(h8v, ya[mi]),
                        part[mi][ni], 0, 0, 0);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                xb[ni] = *reinterpret_cast<const u4v*>(&lds[buf][3][bo + ni * 16 * 64]);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    part[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(h8v, xb[ni]), __builtin_bit_cast(h8v, xa[mi]),
                        part[mi][ni], 0, 0, 0);
            if ((g + 1) % spt == 0) {  // tile column n done: fold with its scales
                const int n = g / spt;
                const int sc = aop.scale(n) + bop.scale(n);
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[mi][ni][v] += ldexpf(part[mi][ni][v], sc);
                        part[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
            if (more) {
                store_pair(&lds[buf ^ 1][0][so], rah);
                store_pair(&lds[buf ^ 1][1][so], ral);
                store_pair(&lds[buf ^ 1][2][so], rbh);
                store_pair(&lds[buf ^ 1][3][so], rbl);
            }
            __syncthreads();
            buf ^= 1;
        }
    }
    double* out = W + rt * (int64_t)nb * nb + (int64_t)bc * kB * nb + br * kB;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * (kB / 2) + mi * 16 + li;
                const int col = wn * (kB / 2) + ni * 16 + 4 * lg + v;
                out[(int64_t)col * nb + row] -= (double)acc[mi][ni][v];
            }
}

// ---------------------------------------------------------------------------
// Wide form of the FP32 / FP16 / BF16 / FP8 groups: 256 x 256 blocks on
// eight waves (2 x 4 waves of 128 x 64), for launches large enough to fill
// the chip with them. Per 64-deep (FP16/BF16; 128 FP8; 32 split) stage a
// block moves half the operand bytes per flop of the 128 x 128 form, and
// each wave reads 1.5x fewer LDS bytes per flop: the 128 x 128 form is
// bound by its operands' path through the vector memory unit and LDS, not
// by the matrix cores. Operands go to a double buffer in LDS through
// registers (wave w fills rows 128 (w & 1) .. + 127 of plane w >> 1;
// planes A0 A1 B0 B1, or A hi, A lo, B hi, B lo for the split; same
// swizzle as above), the next stage's loads in flight under the current
// stage's MFMAs.
// Scales: instead of a second accumulator per tile column, acc holds the
// running sum in units of 2^frame, frame = the current tile column's
// product scale e_a + e_b, and is multiplied by 2^(frame_old - frame_new)
// when the column changes. The block walks its tile columns in ascending
// order of that scale (ties by column), so the frame only rises and acc
// only shrinks: a column's sum is below 2^45 in its own unit (nb <= 4096
// products of at most 2^33), acc stays below Nt 2^45 and never overflows,
// and a rescale is exact unless it drops below binary32's range, which
// only loses terms below 2^-126 of the new unit. (Small terms first is
// also the more accurate order.) One binary32 chain never spans more than
// kWGroup tile columns: the launcher cuts longer ranges at multiples of
// kWGroup columns, and each piece's sum is subtracted from W in binary64,
// so the chains are as long as those of the in-core bulk launches whatever
// the caller's chunking.
constexpr int kWB = 256;              // block rows and columns
constexpr int kWThreads = 512;        // eight waves
constexpr int kWPlane = kWB * 64;     // bytes per plane: 256 rows x 64 bytes
constexpr int kWStage = 4 * kWPlane;  // 64 KiB per stage
constexpr int kWGroup = 16;           // tile columns one binary32 chain may span

template <int MODE>
__global__ __launch_bounds__(kWThreads, 1) void mxp_gemm_wide_kernel(
    double* __restrict__ W, int Nt, int nb, int k, int nbeg, int nend, const int* __restrict__ rows,
    int nrows, const char* __restrict__ storage, const int64_t* __restrict__ shoff,
    const int* __restrict__ cscl) {
    constexpr bool SPLIT = MODE == kFP32;
    constexpr int EB = MODE == kFP8 ? 1 : 2;
    constexpr int SK = SPLIT ? 32 : 128 / EB;  // k per stage
    __shared__ __attribute__((aligned(1024))) uint8_t lds[2 * kWStage];
    __shared__ int key[kWGroup], order[kWGroup];
    const int T = nb / kWB;
    const int64_t total = (int64_t)nrows * T * T;
    const int64_t b = xcd_remap(blockIdx.x, total);
    int64_t rt;
    int br, bc;
    group_block(b, T, false, rows, rt, br, bc);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar load bases
    const int wm = wave & 1, wn = wave >> 1;                     // rows 128 wm, columns 64 wn
    const int li = lane & 15, lg = lane >> 4;
    const NarrowOp aop{storage, shoff, cscl, MODE, Nt, nb, k + rt, (int64_t)br * kWB};
    const NarrowOp bop{storage, shoff, cscl, MODE, Nt, nb, k, (int64_t)bc * kWB};
    const int spt = nb / SK;  // stages per tile column
    const int ncols = nend - nbeg;
    if (ncols > kWGroup) return;  // the launcher never asks for more
    const int g1 = ncols * spt;   // stages, counted from 0
    // tile columns in ascending order of product scale (rank sort)
    for (int c = tid; c < ncols; c += kWThreads) key[c] = aop.scale(nbeg + c) + bop.scale(nbeg + c);
    __syncthreads();
    for (int c = tid; c < ncols; c += kWThreads) {
        const int kc = key[c];
        int r = 0;
        for (int j = 0; j < ncols; ++j) r += (key[j] < kc) || (key[j] == kc && j < c);
        order[r] = c;
    }
    __syncthreads();
    const int pl = wave >> 1, half = wave & 1;
    const int64_t pbyte = SPLIT ? (pl & 1) * (int64_t)nb * nb * 2 : (pl & 1) * 64;
    const int lr = lane >> 2;
    const int lc = (lane & 3) ^ ((lr >> 1) & 3);  // row 16 q + lr swizzles like lr
    const int64_t goff = (int64_t)(128 * half + lr) * nb * EB + 16 * lc + pbyte;
    const int64_t gq = (int64_t)16 * nb * EB;  // 16 rows further
    // the next stage's pieces are loaded into registers while the current
    // stage's MFMAs run, then written to their LDS slots (16 bytes per lane
    // and instruction, lane by lane): on gfx950 this ran 3-12% faster than
    // direct-to-LDS loads into the same slots
    u4v rg[8];
    auto issue = [&](int g) {
        const int c = g / spt, st = g - c * spt;
        const int n = nbeg + order[c];
        const uint8_t* src = (pl < 2 ? aop.rows(n, EB) : bop.rows(n, EB)) + (int64_t)st * SK * EB + goff;
#pragma unroll
        for (int q = 0; q < 8; ++q) rg[q] = *reinterpret_cast<const u4v*>(src + q * gq);
    };
    auto commit = [&](int g) {
        uint8_t* dst = lds + (g & 1) * kWStage + pl * kWPlane + half * 128 * 64 + lane * 16;
#pragma unroll
        for (int q = 0; q < 8; ++q) *reinterpret_cast<u4v*>(dst + q * 1024) = rg[q];
    };
    const int ro = swz(li, lg);
    f4 acc[8][4];
#pragma unroll
    for (int mi = 0; mi < 8; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
    // this lane's first output element; the others are uniform offsets from it
    double* const out = W + rt * (int64_t)nb * nb + (int64_t)(bc * kWB + wn * 64 + 4 * lg) * nb +
                        br * kWB + wm * 128 + li;
    int frame = 0;
    if (g1 > 0) {
        frame = key[order[0]];
        issue(0);
        commit(0);
    }
    for (int g = 0; g < g1; ++g) {
        // stage g is in LDS for every wave, and every wave is done reading
        // stage g - 1's buffer, which stage g + 1 overwrites below
        __syncthreads();
        if (g + 1 < g1) issue(g + 1);
        const uint8_t* st = lds + (g & 1) * kWStage;
        const int ao = wm * 128 * 64 + ro, bo = wn * 64 * 64 + ro;
        if constexpr (SPLIT) {
            u4v xa[8], xb[4], ya[8];
#pragma unroll
            for (int mi = 0; mi < 8; ++mi) xa[mi] = *reinterpret_cast<const u4v*>(st + ao + mi * 1024);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                xb[ni] = *reinterpret_cast<const u4v*>(st + 2 * kWPlane + bo + ni * 1024);
#pragma unroll
            for (int mi = 0; mi < 8; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(h8v, xb[ni]), __builtin_bit_cast(h8v, xa[mi]), acc[mi][ni],
                        0, 0, 0);
#pragma unroll
            for (int mi = 0; mi < 8; ++mi)
                ya[mi] = *reinterpret_cast<const u4v*>(st + kWPlane + ao + mi * 1024);
#pragma unroll
            for (int mi = 0; mi < 8; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(h8v, xb[ni]), __builtin_bit_cast(h8v, ya[mi]), acc[mi][ni],
                        0, 0, 0);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                xb[ni] = *reinterpret_cast<const u4v*>(st + 3 * kWPlane + bo + ni * 1024);
#pragma unroll
            for (int mi = 0; mi < 8; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(h8v, xb[ni]), __builtin_bit_cast(h8v, xa[mi]), acc[mi][ni],
                        0, 0, 0);
        } else if constexpr (MODE == kFP8) {
            // lane group l / 16 takes chunk l / 16 of both planes (32 k)
            i8v bq[4];
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const u4v x = *reinterpret_cast<const u4v*>(st + 2 * kWPlane + bo + ni * 1024);
                const u4v y = *reinterpret_cast<const u4v*>(st + 3 * kWPlane + bo + ni * 1024);
                bq[ni] = i8v{(int)x.x, (int)x.y, (int)x.z, (int)x.w, (int)y.x, (int)y.y, (int)y.z, (int)y.w};
            }
#pragma unroll
            for (int mi = 0; mi < 8; ++mi) {
                const u4v x = *reinterpret_cast<const u4v*>(st + ao + mi * 1024);
                const u4v y = *reinterpret_cast<const u4v*>(st + kWPlane + ao + mi * 1024);
                const i8v a = i8v{(int)x.x, (int)x.y, (int)x.z, (int)x.w, (int)y.x, (int)y.y, (int)y.z, (int)y.w};
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        bq[ni], a, acc[mi][ni], 0, 0, 0, 127, 0, 127);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {  // plane ks: k 32 ks .. 32 ks + 31
                u4v a[8], bq[4];
#pragma unroll
                for (int mi = 0; mi < 8; ++mi)
                    a[mi] = *reinterpret_cast<const u4v*>(st + ks * kWPlane + ao + mi * 1024);
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    bq[ni] = *reinterpret_cast<const u4v*>(st + (2 + ks) * kWPlane + bo + ni * 1024);
#pragma unroll
                for (int mi = 0; mi < 8; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni) {
                        if constexpr (MODE == kFP16)
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                __builtin_bit_cast(h8v, bq[ni]), __builtin_bit_cast(h8v, a[mi]),
                                acc[mi][ni], 0, 0, 0);
                        else
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(b8v, bq[ni]), __builtin_bit_cast(b8v, a[mi]),
                                acc[mi][ni], 0, 0, 0);
                    }
            }
        }
        if (g + 1 < g1) commit(g + 1);
        if (g + 1 < g1 && (g + 1) % spt == 0) {  // the next stage starts a tile column
            const int sc = key[order[(g + 1) / spt]];
            const int d = frame - sc;  // <= 0: the frame rises
            if (d != 0) {
#pragma unroll
                for (int mi = 0; mi < 8; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[mi][ni][v] = ldexpf(acc[mi][ni][v], d);
            }
            frame = sc;
        }
    }
    // W -= acc 2^frame for this wave's 128 x 64 part
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double* const p = out + (int64_t)(ni * 16 + v) * nb;
#pragma unroll
            for (int mi = 0; mi < 8; ++mi) p[mi * 16] -= ldexp((double)acc[mi][ni][v], frame);
        }
}

// Wide form for this group launch? mode 1: whenever the tile allows it;
// -1: never; 0: when the launch has at least 128 blocks, half a block per
// CU (threshold measured on the n = 131072 mixed factorization against 1,
// 64, 256, 512 and 1024 blocks; with the register-staged loads 128 was
// 0.6% faster than 256 with binary64 updates into FP64 tiles and equal
// with FP32-class updates, and 64 was slower).
bool use_wide(int mode, int nb, int nrows) {
    if (mode < 0 || nb % kWB != 0) return false;
    const int64_t T = nb / kWB;
    return mode > 0 || (int64_t)nrows * T * T >= 128;
}

}  // namespace

// Split count of an FP64 group launch: the forward panel's time model
// (rounds of 256 workgroups at the FP64 MFMA rate, plus the partial
// blocks' traffic; counting the two resident workgroups per CU as 512
// slots measured no faster), each split keeping >= 1024 of K and the
// partials within `cap` doubles.
static int mxp_f64_splits(int64_t nblocks, int64_t K, size_t cap) {
    int64_t smax = K / 1024;
    if (smax > 16) smax = 16;
    while (smax > 1 && (size_t)smax * nblocks * kB * kB > cap) --smax;
    if (smax <= 1) return 1;
    const int64_t slots = 256;
    const double slot_flops = 78.6e12 / slots;
    const double blk_bytes = (double)kB * kB * sizeof(double);
    double best = 1e300;
    int bests = 1;
    for (int64_t s = 1; s <= smax; ++s) {
        const double rounds = (double)((nblocks * s + slots - 1) / slots);
        double t = rounds * (2.0 * kB * kB * ((double)K / s)) / slot_flops;
        if (s > 1) t += 3.0 * s * nblocks * blk_bytes / 5e12;
        if (t < best * 0.97) {
            best = t;
            bests = (int)s;
        }
    }
    return bests;
}

hipError_t launch_mxp_gemm_f64(hipStream_t s, double* W, int Nt, int nb, int k, int nbeg, int nend,
                               const int* rows, int nrows, bool diag, const char* storage,
                               const int64_t* toff, const uint8_t* tcls, const int* tscl,
                               double* partial, size_t partial_cap) {
    const int64_t T = nb / kB;
    const int64_t total = (diag ? T * (T + 1) / 2 : 0) + (int64_t)nrows * T * T;
    if (total == 0 || nend <= nbeg) return hipSuccess;
    const int64_t K0 = (int64_t)nbeg * nb, K1 = (int64_t)nend * nb, K = K1 - K0;
    const int splits = mxp_f64_splits(total, K, partial_cap);
    const int64_t kchunk = (((K + splits - 1) / splits + 15) / 16) * 16;
    hipLaunchKernelGGL(mxp_gemm_f64_kernel, dim3((unsigned)(total * splits)), dim3(kF64Threads), 0,
                       s, W, Nt, nb, k, K0, K1, rows, nrows, diag ? 1 : 0, storage, toff, tcls, tscl,
                       splits, kchunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    hipLaunchKernelGGL(mxp_group_reduce_kernel, dim3((unsigned)total), dim3(256), 0, s, W, nb, rows,
                       diag ? 1 : 0, total, splits, partial);
    return hipGetLastError();
}

hipError_t launch_mxp_gemm_f32(hipStream_t s, double* W, int Nt, int nb, int k, int nbeg, int nend,
                               const int* rows, int nrows, const char* storage,
                               const int64_t* shoff, const int* cscl, int wide) {
    if (nrows <= 0 || nend <= nbeg) return hipSuccess;
    if (use_wide(wide, nb, nrows)) {
        const int64_t T = nb / kWB;
        for (int p0 = nbeg; p0 < nend;) {  // pieces cut at multiples of kWGroup columns
            const int p1 = std::min(nend, (p0 / kWGroup + 1) * kWGroup);
            hipLaunchKernelGGL(mxp_gemm_wide_kernel<kFP32>, dim3((unsigned)(nrows * T * T)),
                               dim3(kWThreads), 0, s, W, Nt, nb, k, p0, p1, rows, nrows, storage,
                               shoff, cscl);
            if (hipError_t e = hipGetLastError()) return e;
            p0 = p1;
        }
        return hipSuccess;
    }
    const int64_t T = nb / kB;
    const int64_t total = (int64_t)nrows * T * T;
    hipLaunchKernelGGL(mxp_gemm_split_kernel, dim3((unsigned)total), dim3(kGemmThreads), 0, s, W,
                       Nt, nb, k, nbeg, nend, rows, nrows, storage, shoff, cscl);
    return hipGetLastError();
}

hipError_t launch_mxp_gemm_narrow(hipStream_t s, double* W, int Nt, int nb, int k, int nbeg,
                                  int nend, const int* rows, int nrows, int cls,
                                  const char* storage, const int64_t* shoff, const int* cscl,
                                  int wide) {
    if (nrows <= 0 || nend <= nbeg) return hipSuccess;
    if (use_wide(wide, nb, nrows)) {
        if (cls != kFP16 && cls != kBF16 && cls != kFP8) return hipErrorInvalidValue;
        const int64_t T = nb / kWB;
        const dim3 grid((unsigned)(nrows * T * T)), block(kWThreads);
        for (int p0 = nbeg; p0 < nend;) {  // pieces cut at multiples of kWGroup columns
            const int p1 = std::min(nend, (p0 / kWGroup + 1) * kWGroup);
            if (cls == kFP16)
                hipLaunchKernelGGL(mxp_gemm_wide_kernel<kFP16>, grid, block, 0, s, W, Nt, nb, k,
                                   p0, p1, rows, nrows, storage, shoff, cscl);
            else if (cls == kBF16)
                hipLaunchKernelGGL(mxp_gemm_wide_kernel<kBF16>, grid, block, 0, s, W, Nt, nb, k,
                                   p0, p1, rows, nrows, storage, shoff, cscl);
            else
                hipLaunchKernelGGL(mxp_gemm_wide_kernel<kFP8>, grid, block, 0, s, W, Nt, nb, k,
                                   p0, p1, rows, nrows, storage, shoff, cscl);
            if (hipError_t e = hipGetLastError()) return e;
            p0 = p1;
        }
        return hipSuccess;
    }
    const int64_t T = nb / kB;
    const int64_t total = (int64_t)nrows * T * T;
    const dim3 grid((unsigned)total), block(kGemmThreads);
    if (cls == kFP16)
        hipLaunchKernelGGL(mxp_gemm_narrow_kernel<kFP16>, grid, block, 0, s, W, Nt, nb, k, nbeg, nend,
                           rows, nrows, storage, shoff, cscl);
    else if (cls == kBF16)
        hipLaunchKernelGGL(mxp_gemm_narrow_kernel<kBF16>, grid, block, 0, s, W, Nt, nb, k, nbeg, nend,
                           rows, nrows, storage, shoff, cscl);
    else if (cls == kFP8)
        hipLaunchKernelGGL(mxp_gemm_narrow_kernel<kFP8>, grid, block, 0, s, W, Nt, nb, k, nbeg, nend,
                           rows, nrows, storage, shoff, cscl);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_mxp_copies(hipStream_t s, int nb, const int* list, int count, char* storage,
                             const int64_t* toff, const uint8_t* tcls, const int* tscl,
                             const int64_t* shoff, const int* cscl) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(tile_copies_kernel, dim3(nb / kCB, nb / kCB, count), dim3(kThreads), 0, s, nb,
                       list, storage, toff, tcls, tscl, shoff, cscl);
    return hipGetLastError();
}

hipError_t launch_slot_tables(hipStream_t s, const int64_t* upd, int count, const uint8_t* need,
                              const int64_t* coff, int64_t* toff, int64_t* shoff) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(slot_tables_kernel, dim3((count + 255) / 256), dim3(256), 0, s, upd, count,
                       need, coff[0], coff[1], coff[2], coff[3], toff, shoff);
    return hipGetLastError();
}

hipError_t launch_mxp_finalize(hipStream_t s, const double* W, int Nt, int nb, int k, double* part,
                               char* storage, const int64_t* toff, const uint8_t* tcls, int* tscl,
                               const int64_t* shoff, int* cscl) {
    const int rows = Nt - k - 1;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(tile_amax_kernel, dim3(kStrips, rows), dim3(kThreads), 0, s,
                       W + (int64_t)nb * nb, nb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tile_cast_kernel, dim3(nb / kCB, nb / kCB, rows), dim3(kThreads), 0, s, W, Nt,
                       nb, k, part, storage, toff, tcls, tscl, shoff, cscl);
    return hipGetLastError();
}

}  // namespace tc
