// The pair sweep for wide points (65 to 4096 coordinates, bf16 or fp16
// operands): the product A p of Algorithm 1 without a stored kernel matrix
// when the distance contraction, not the kernel evaluation, dominates the
// pair cost (2 (d + 6) MFMA flops against ~10 VALU slots per pair).
//
// The same 256-point block pairs and partial layout as the narrow sweep
// (matvec.hip), so the product is finished by the same kernels, under a
// tiled schedule (wide_plan): a work item (one 512-thread workgroup, eight
// waves) takes a row block I of a group of eight and every fourth block
// offset of a range, so that the 32 items of a tile, run together on one
// XCD, touch eight row and four column blocks at a time and share them in
// its L2.  For each block pair (I, J) the augmented operands of both blocks
// stream through LDS in 32-element slices of K (four stages: the pair's
// first three by direct global-to-LDS loads, the rest loaded into registers
// three stages ahead and written to LDS a stage later), each wave
// accumulating a 64 x 128 part of the 256 x 256 distance tile in eight
// 32x32x16 MFMA tiles; the two halves of the waves run a phase apart, so
// that on each SIMD one wave multiplies while the other reads LDS.  The
// slices are stored with the 16-byte groups of a row XOR-swizzled by the row
// index, so that the rows a fragment read serves together fall in distinct
// LDS banks.  After the last slice the kernel values are formed in registers
// on the MFMA output layout and folded into FP32 row sums (added across the
// lanes after each block pair, into LDS) and per-block-pair column sums.
#include <algorithm>
#include <cmath>

#include "blas.h"
#include "host.h"
#include "sweep.h"

namespace dcg {

constexpr int kWideRows = 256;  // points per block (rows and columns)
constexpr int kWideKC = 32;     // K elements per LDS stage (two MFMA K-steps)
constexpr int kWideSlots = kWideRows * 4;   // 16-byte slots of one operand in a stage

// s_waitcnt immediates that wait for the vector-memory counter only
// (vmcnt in bits 3:0, expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
constexpr int kVmcnt0 = 0xF70, kVmcnt4 = 0xF74, kVmcnt8 = 0xF78;
// ... and the one that waits for the LDS / scalar-memory counter only
// (lgkmcnt 0, vmcnt and expcnt at their maxima)
constexpr int kLgkm0 = 0xC07F;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void global_void;

template <int OPK>
__device__ __forceinline__ f32x16 wide_mfma(const u32x4 &a, const u32x4 &b, const f32x16 &c) {
  if constexpr (OPK == kOpF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// A barrier for LDS traffic only: this wave's LDS accesses are complete
// (lgkmcnt), the global loads in flight are not waited for (the release
// fence of __syncthreads would); the empty asm statements keep the compiler
// from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(kLgkm0);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The value of lane l ^ D (D < 32) by a swizzle within each 32 lanes
// (bit-mask mode: and-mask 31, xor-mask D).
template <int D>
__device__ __forceinline__ float lane_xor(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), 0x1F | (D << 10)));
}

// Steps per row block group of the tiled schedule (as wide_steps on the
// host).
__device__ __forceinline__ int wide_steps_dev(int nb) { return (nb / 2 + 1 + kWideGroup - 1 + 3) / 4; }

// Slot of the 16-byte group g (0..3) of row `row` in a stage (64-byte rows).
// A fragment read takes group g of 32 consecutive rows, served 16 lanes at a
// time over 256 bytes of banks: rows r and r + 4 share those bytes' quarter,
// so the group is XOR-ed with bits 2-3 of the row and any 16 consecutive
// rows use 16 distinct 16-byte bank groups.
__device__ __forceinline__ int wide_slot(int row, int g) {
  return row * 4 + (g ^ ((row >> 2) & 3));
}

template <int KERN, int OPK>
__global__ __launch_bounds__(512, 1) void symv_wide_kernel(SymvArgs A) {
  if (A.done != nullptr && *A.done != 0) return;
  // Tiles are dealt to the XCDs round-robin (workgroup w goes to XCD w mod
  // 8), each XCD running its tiles' 32 work items back to back, so that the
  // items that share a tile's blocks share an L2.
  const int nb = A.nb;
  const int parts = A.nchunk / 4;
  const int64_t tiles = int64_t((nb + kWideGroup - 1) / kWideGroup) * parts;
  const int64_t j = blockIdx.x >> 3;
  const int64_t tile = (j >> 5) * 8 + (blockIdx.x & 7);
  if (tile >= tiles) return;
  const int grp = static_cast<int>(tile / parts), part = static_cast<int>(tile % parts);
  const int ia = static_cast<int>((j & 31) >> 2), ib = static_cast<int>(j & 3);
  const int I = kWideGroup * grp + ia;
  if (I >= nb) return;
  const int ndel = ((nb % 2) == 0 && I >= nb / 2) ? A.dmax : A.dmax + 1;
  const int s0 = part * A.chunk;
  const int s1 = min(s0 + A.chunk, wide_steps_dev(nb));
  const int c = 4 * part + ib;   // this item's row-partial slot

  const int tid = threadIdx.x;
  // the wave index as a scalar (it is uniform), so that the extra barriers
  // of the two wave groups below are scalar branches
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l = tid & 63, lc = l & 31, lh = l >> 5;
  const int wr = w & 3, wc = w >> 2;     // rows 64 wr .., columns 128 wc .. of a block pair
  const int64_t n_pad = A.n_pad;
  const int kst = A.kstride;             // a multiple of kWideKC
  const int nkc = kst / kWideKC;

  // four stages: slots [0, kWideSlots) the row block's operand, the rest
  // the column block's
  __shared__ u32x4 St0[2 * kWideSlots];
  __shared__ u32x4 St1[2 * kWideSlots];
  __shared__ u32x4 St2[2 * kWideSlots];
  __shared__ u32x4 St3[2 * kWideSlots];
  __shared__ float rowacc[2][kWideRows];
  __shared__ float colpart[4][kWideRows];
  __shared__ __attribute__((aligned(16))) float vrow[kWideRows];   // the input vector on this row block
  __shared__ float vcol[2][kWideRows];   // ... on the column blocks of two pairs

  for (int e = tid; e < 2 * kWideRows; e += 512) rowacc[e / kWideRows][e % kWideRows] = 0.0f;
  for (int e = tid; e < kWideRows; e += 512) vrow[e] = A.vin[int64_t(I) * kWideRows + e];
  __syncthreads();

  const uint16_t *xr = static_cast<const uint16_t *>(A.xr);
  const uint16_t *xc = static_cast<const uint16_t *>(A.xc);
  // Loads: a stage is 32 chunks of 1 KB (64 slots), lane l of a load
  // writing slot 64 (chunk) + l (directly or from a staging register).
  // Waves 0-3 load the row block's operand (chunks 4 wr + i, i < 4), waves
  // 4-7 the column block's; a lane fetches the row and group its slot holds.
  const int opsel = wc;
  int go0, go1, go2, go3;                // element offsets within the block
  {
    int s = (4 * wr + 0) * 64 + l, row = s >> 2;
    go0 = row * kst + 8 * ((s & 3) ^ ((row >> 2) & 3));
    s = (4 * wr + 1) * 64 + l; row = s >> 2;
    go1 = row * kst + 8 * ((s & 3) ^ ((row >> 2) & 3));
    s = (4 * wr + 2) * 64 + l; row = s >> 2;
    go2 = row * kst + 8 * ((s & 3) ^ ((row >> 2) & 3));
    s = (4 * wr + 3) * 64 + l; row = s >> 2;
    go3 = row * kst + 8 * ((s & 3) ^ ((row >> 2) & 3));
  }
  const int dst0 = opsel * kWideSlots + (4 * wr) * 64;   // this wave's first chunk

#define DCG_WIDE_ISSUE(BUF, kc)                                                              \
  do {                                                                                       \
    const uint16_t *src = base + (kc) * kWideKC;                                             \
    __builtin_amdgcn_global_load_lds((global_void *)(src + go0), (lds_void *)&BUF[dst0], 16, \
                                     0, 0);                                                  \
    __builtin_amdgcn_global_load_lds((global_void *)(src + go1),                             \
                                     (lds_void *)&BUF[dst0 + 64], 16, 0, 0);                 \
    __builtin_amdgcn_global_load_lds((global_void *)(src + go2),                             \
                                     (lds_void *)&BUF[dst0 + 128], 16, 0, 0);                \
    __builtin_amdgcn_global_load_lds((global_void *)(src + go3),                             \
                                     (lds_void *)&BUF[dst0 + 192], 16, 0, 0);                \
  } while (0)
#define DCG_WIDE_MFMAS(a0, a1, b0, b1, b2, b3)                                               \
  acc[0][0] = wide_mfma<OPK>(a0, b0, acc[0][0]);                                             \
  acc[0][1] = wide_mfma<OPK>(a0, b1, acc[0][1]);                                             \
  acc[0][2] = wide_mfma<OPK>(a0, b2, acc[0][2]);                                             \
  acc[0][3] = wide_mfma<OPK>(a0, b3, acc[0][3]);                                             \
  acc[1][0] = wide_mfma<OPK>(a1, b0, acc[1][0]);                                             \
  acc[1][1] = wide_mfma<OPK>(a1, b1, acc[1][1]);                                             \
  acc[1][2] = wide_mfma<OPK>(a1, b2, acc[1][2]);                                             \
  acc[1][3] = wide_mfma<OPK>(a1, b3, acc[1][3])
  // Inside the stage loop the loads go through registers (four 16-byte
  // groups per lane, written to LDS a stage later): the direct loads' writes
  // into LDS held the LDS for longer than register-staged writes do.  The
  // direct loads remain for each pair's first three stages, which load
  // during the previous pair's epilogue.
  u32x4 rs0, rs1, rs2, rs3;
#define DCG_WIDE_LOADR(kc)                                                                   \
  do {                                                                                       \
    const uint16_t *src = base + (kc) * kWideKC;                                             \
    rs0 = *reinterpret_cast<const u32x4 *>(src + go0);                                       \
    rs1 = *reinterpret_cast<const u32x4 *>(src + go1);                                       \
    rs2 = *reinterpret_cast<const u32x4 *>(src + go2);                                       \
    rs3 = *reinterpret_cast<const u32x4 *>(src + go3);                                       \
  } while (0)
#define DCG_WIDE_STORER(BUF)                                                                 \
  do {                                                                                       \
    BUF[dst0 + l] = rs0;                                                                     \
    BUF[dst0 + 64 + l] = rs1;                                                                \
    BUF[dst0 + 128 + l] = rs2;                                                               \
    BUF[dst0 + 192 + l] = rs3;                                                               \
  } while (0)
  // fragments of both K-steps of a stage (16-byte groups lh and 2 + lh of
  // this wave's two 32-row and four 32-column tiles)
  u32x4 fa0, fa1, fb0, fb1, fb2, fb3, ga0, ga1, gb0, gb1, gb2, gb3;
#define DCG_WIDE_READ(BUF)                                                                   \
  do {                                                                                       \
    fa0 = BUF[wide_slot(64 * wr + lc, lh)];                                                  \
    fa1 = BUF[wide_slot(64 * wr + 32 + lc, lh)];                                             \
    fb0 = BUF[kWideSlots + wide_slot(128 * wc + lc, lh)];                                    \
    fb1 = BUF[kWideSlots + wide_slot(128 * wc + 32 + lc, lh)];                               \
    fb2 = BUF[kWideSlots + wide_slot(128 * wc + 64 + lc, lh)];                               \
    fb3 = BUF[kWideSlots + wide_slot(128 * wc + 96 + lc, lh)];                               \
    ga0 = BUF[wide_slot(64 * wr + lc, 2 + lh)];                                              \
    ga1 = BUF[wide_slot(64 * wr + 32 + lc, 2 + lh)];                                         \
    gb0 = BUF[kWideSlots + wide_slot(128 * wc + lc, 2 + lh)];                                \
    gb1 = BUF[kWideSlots + wide_slot(128 * wc + 32 + lc, 2 + lh)];                           \
    gb2 = BUF[kWideSlots + wide_slot(128 * wc + 64 + lc, 2 + lh)];                           \
    gb3 = BUF[kWideSlots + wide_slot(128 * wc + 96 + lc, 2 + lh)];                           \
  } while (0)
#define DCG_WIDE_MULT()                                                                      \
  do {                                                                                       \
    DCG_WIDE_MFMAS(fa0, fa1, fb0, fb1, fb2, fb3);                                            \
    DCG_WIDE_MFMAS(ga0, ga1, gb0, gb1, gb2, gb3);                                            \
  } while (0)
// Stage s in buffer CUR: write the staged stage s + 2 (loaded a stage ago)
// to W2 (stage s - 2's buffer), load stage s + 3 into the staging
// registers, read the stage's fragments, barrier, multiply, barrier.  The
// waves of group 1 (columns 128-255 of the pair) pass one barrier more
// before the stage loop and those of group 0 one more after it, so group 1
// runs a phase behind: while group 0 multiplies stage s, group 1 reads it,
// and while group 0 reads stage s + 1, group 1 multiplies s.  Each SIMD
// holds one wave of each group, so one of its waves issues MFMAs while the
// other reads LDS.  W2 is free: both groups read stage s - 2 at least two
// phases ago; stage s + 2 is read after the barriers that follow both
// groups' writes of it (each barrier waits for this wave's LDS accesses).
// Plain s_barriers: the release fence of __syncthreads would wait for the
// loads in flight too.  The MFMAs touch no memory, so scheduling barriers
// keep them between the two workgroup barriers; the multiplying wave runs at
// the higher issue priority.
#define DCG_WIDE_STAGE(CUR, W2, s)                                                           \
  do {                                                                                       \
    if ((s) >= 1 && (s) + 2 < nkc) {                                                         \
      __builtin_amdgcn_s_waitcnt(kVmcnt0);                                                   \
      DCG_WIDE_STORER(W2);                                                                   \
    }                                                                                        \
    if ((s) + 3 < nkc) DCG_WIDE_LOADR((s) + 3);                                              \
    DCG_WIDE_READ(CUR);                                                                      \
    lds_barrier();                                                                           \
    __builtin_amdgcn_sched_barrier(0);                                                       \
    __builtin_amdgcn_s_setprio(1);                                                           \
    DCG_WIDE_MULT();                                                                         \
    __builtin_amdgcn_s_setprio(0);                                                           \
    __builtin_amdgcn_sched_barrier(0);                                                       \
    lds_barrier();                                                                           \
  } while (0)

  // the first step at or after st whose pair this item owns (s1 if none)
  auto next_valid = [&](int st) {
    for (; st < s1; ++st) {
      const int u = 4 * st + ib - ia;
      if (u >= 0 && u < ndel) break;
    }
    return st;
  };
  auto base_of = [&](int st) {
    int J = I + 4 * st + ib - ia;
    if (J >= nb) J -= nb;
    return opsel == 0 ? xr + int64_t(I) * kWideRows * kst : xc + int64_t(J) * kWideRows * kst;
  };
  // the input vector on a pair's column block, loaded into vcol[b] by
  // direct global-to-LDS loads (waves 0-3, 64 entries each) when the pair's
  // first stages are issued: it has landed by the pair's first stage wait
  auto issue_vcol = [&](int b, int st) {
    int J = I + 4 * st + ib - ia;
    if (J >= nb) J -= nb;
    if (w < 4)
      __builtin_amdgcn_global_load_lds((global_void *)(A.vin + int64_t(J) * kWideRows + 64 * w + l),
                                       (lds_void *)&vcol[b][64 * w], 4, 0, 0);
  };
  int pb = 0;
  int st = next_valid(s0);
  const uint16_t *base = nullptr;
  if (st < s1) {
    issue_vcol(0, st);
    base = base_of(st);
    DCG_WIDE_ISSUE(St0, 0);
    if (1 < nkc) DCG_WIDE_ISSUE(St1, 1);
    if (2 < nkc) DCG_WIDE_ISSUE(St2, 2);
  }
  while (st < s1) {
    const int dl = 4 * st + ib - ia;   // block offset of this step's pair
    int J = I + dl;
    if (J >= nb) J -= nb;
    f32x16 acc[2][4];
#pragma unroll
    for (int tr = 0; tr < 2; ++tr)
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) acc[tr][tc] = f32x16{};
    // everything this pair's first stages need has landed (and the
    // previous pair's stores, which may retire out of order with loads)
    __builtin_amdgcn_s_waitcnt(kVmcnt0);
    lds_barrier();
    if (wc != 0) lds_barrier();   // group 1 one phase behind
    for (int kc = 0; kc < nkc; kc += 4) {
      DCG_WIDE_STAGE(St0, St2, kc);
      if (kc + 1 < nkc) DCG_WIDE_STAGE(St1, St3, kc + 1);
      if (kc + 2 < nkc) DCG_WIDE_STAGE(St2, St0, kc + 2);
      if (kc + 3 < nkc) DCG_WIDE_STAGE(St3, St1, kc + 3);
    }
    if (wc == 0) lds_barrier();   // ... and level again: every wave is done
    // this pair's column-block vector, read while no direct load is in
    // flight (the compiler would otherwise wait for the next pair's)
    float pj[4];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) pj[tc] = vcol[pb][128 * wc + 32 * tc + lc];
    // every wave is done reading this pair's stages (the last barrier): the
    // next pair's first three stages load while this pair's epilogue runs
    const int stn = next_valid(st + 1);
    if (stn < s1) {
      issue_vcol(pb ^ 1, stn);
      base = base_of(stn);
      DCG_WIDE_ISSUE(St0, 0);
      if (1 < nkc) DCG_WIDE_ISSUE(St1, 1);
      if (2 < nkc) DCG_WIDE_ISSUE(St2, 2);
    }
#undef DCG_WIDE_ISSUE
#undef DCG_WIDE_READ
#undef DCG_WIDE_MFMAS
#undef DCG_WIDE_MULT
#undef DCG_WIDE_STAGE
#undef DCG_WIDE_LOADR
#undef DCG_WIDE_STORER

    // kernel values on the MFMA output layout: lane l holds column l % 32
    // and rows 8 (v / 4) + 4 (l / 32) + v % 4 of each 32x32 tile; the row
    // sums stay per lane (over the lane's columns) for all of the work
    // item's block pairs and are added across lanes once at its end
    const bool diag = (dl == 0);

    // the exact diagonal of the diagonal block pair: distance zero by
    // definition (a wave-uniform test per tile)
    if (diag) {
#pragma unroll
      for (int tr = 0; tr < 2; ++tr)
#pragma unroll
        for (int tc = 0; tc < 4; ++tc)
          if (2 * wr + tr == 4 * wc + tc) {
#pragma unroll
            for (int v = 0; v < 16; ++v)
              if (8 * (v >> 2) + 4 * lh + (v & 3) == lc) acc[tr][tc][v] = 0.0f;
          }
    }
    // row sums per lane, and column sums (used off the diagonal block pair,
    // where the row sums alone cover both triangles)
    float cs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int tr = 0; tr < 2; ++tr) {
      // the lane's 16 rows of this tile row: four runs of four (16-byte reads)
      f32x4 vi[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        vi[q] = *reinterpret_cast<const f32x4 *>(&vrow[64 * wr + 32 * tr + 8 * q + 4 * lh]);
      float rs[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) rs[v] = 0.0f;
#pragma unroll
      for (int tc = 0; tc < 4; ++tc)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float kv = kval<KERN>(acc[tr][tc][v]);
          rs[v] = fmaf(kv, pj[tc], rs[v]);
          cs[tc] = fmaf(kv, vi[v >> 2][v & 3], cs[tc]);
        }
      // the sums of the 16 rows over the 32 lanes of this lane's half: four
      // halving exchanges leave entry lc / 2 summed over 16 lanes, the last
      // one over all 32; lane pairs then add it to the row's LDS sum
#define DCG_WIDE_HALVE(D, M)                                                                 \
      {                                                                                      \
        const bool hi = (lc & (D)) != 0;                                                     \
        _Pragma("unroll") for (int i = 0; i < (M); ++i) {                                    \
          const float keep = hi ? rs[(M) + i] : rs[i];                                       \
          const float send = hi ? rs[i] : rs[(M) + i];                                       \
          rs[i] = keep + lane_xor<(D)>(send);                                                \
        }                                                                                    \
      }
      DCG_WIDE_HALVE(16, 8);
      DCG_WIDE_HALVE(8, 4);
      DCG_WIDE_HALVE(4, 2);
      DCG_WIDE_HALVE(2, 1);
#undef DCG_WIDE_HALVE
      const float rsum = rs[0] + lane_xor<1>(rs[0]);
      if ((lc & 1) == 0) {
        const int v = lc >> 1;
        rowacc[wc][64 * wr + 32 * tr + 8 * (v >> 2) + 4 * lh + (v & 3)] += rsum;
      }
    }
    // column sums of an off-diagonal block pair: the block's four row
    // quarters added in a fixed order
    if (!diag) {
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) {
        const float s = cs[tc] + __shfl_xor(cs[tc], 32);
        if (lh == 0) colpart[wr][128 * wc + 32 * tc + lc] = s;
      }
      lds_barrier();
      for (int e = tid; e < kWideRows; e += 512) {
        const float s = (colpart[0][e] + colpart[1][e]) + (colpart[2][e] + colpart[3][e]);
        A.pcol[int64_t(dl - 1) * n_pad + int64_t(J) * kWideRows + e] = s;
      }
      lds_barrier();
    }
    st = stn;
    pb ^= 1;
  }
  __syncthreads();
  for (int e = tid; e < kWideRows; e += 512)
    A.prow[int64_t(c) * n_pad + int64_t(I) * kWideRows + e] =
        static_cast<double>(rowacc[0][e]) + static_cast<double>(rowacc[1][e]);
}

template <int OPK>
static void launch_wide_kernel(int kernel, const SymvArgs &a, int64_t grid, hipStream_t s) {
  const dim3 g(static_cast<unsigned>(grid)), b(512);
  if (kernel == DCG_RBF) hipLaunchKernelGGL((symv_wide_kernel<DCG_RBF, OPK>), g, b, 0, s, a);
  else if (kernel == DCG_MATERN32)
    hipLaunchKernelGGL((symv_wide_kernel<DCG_MATERN32, OPK>), g, b, 0, s, a);
  else hipLaunchKernelGGL((symv_wide_kernel<DCG_MATERN52, OPK>), g, b, 0, s, a);
}

int launch_symv_wide(const dcg_operator_s *op, const SymvArgs &a, int64_t grid) {
  const Geometry &g = op->g;
  if (!sweep_wide(g) || g.kstride % kWideKC != 0 || sweep_blk(g, 1) != kWideRows ||
      g.n_pad % kWideRows != 0 || grid < 256 || grid % 256 != 0 || a.nchunk % 4 != 0)
    return DCG_E_ARG;
  if (g.opk == kOpF16) launch_wide_kernel<kOpF16>(op->kernel, a, grid, op->stream);
  else launch_wide_kernel<kOpBf16>(op->kernel, a, grid, op->stream);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

}  // namespace dcg
