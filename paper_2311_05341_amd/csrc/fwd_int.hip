// Integer forward kernels (uint8, packed uint4 and uint16 input) for gfx950.
//
// Forward transform, Sec. 2, Eq. 3:  S(d, t) = sum_c x(c, t + shift(c, d)).
//
// Tiling.  A workgroup of NW waves owns NW*R consecutive DM rows (a "DM block")
// and 64*NS consecutive output samples (a "time tile"); wave w owns R of the
// rows and each lane NS of their samples (NS/4 words of 4 samples, strided by
// 64 words so that the wave's LDS accesses are contiguous), in registers.
// Channels are visited in blocks of `chan_block`: the rows of a channel block
// are staged in LDS once, starting at the block's first-DM delay rounded down
// to 16 bytes, and each staged sample then serves all NW*R DM rows of the
// workgroup (the data reuse of the shared-memory algorithm of Sec. 4.1).  Two
// LDS buffers alternate.
//
// Byte alignment.  LDS reads on gfx950 are fast only when naturally aligned,
// but a DM's delay starts its window at any byte.  Each staged row is therefore
// kept in four copies shifted by 0..3 bytes ("phases").  For a (channel, DM)
// pair with window offset o, a lane reads the copy of phase o % 4 from byte
// o - o % 4 on: whole, aligned 32-bit words, no realignment arithmetic.
//
// Exact arithmetic with two samples per add (the SIMD-within-a-word idea of
// Sec. 4.1).  For each 4-sample word w = [b0 b1 b2 b3] a lane adds
//     mix += w                       (all four bytes; carries cross byte lanes)
//     odd += [b1, 0, b3, 0]          (two 16-bit lanes, one v_perm)
// For <= 257 channels no 16-bit lane of `odd` overflows, and
//     mix - (odd << 8) = sum b0 + 2^16 * sum b2        (mod 2^32)
// recovers the even samples exactly.  Every 256 channels both are flushed into
// per-sample int32 totals, which stay below 2^24 and convert to float exactly.
//
// 16-bit input.  A word holds two samples; a 16-bit window starts on an even
// byte, so two copies (shifted by 0 and 2 bytes) align every window.  Per word
// w = [lo hi] a lane adds
//     mix += w          (the low half carries into the high half)
//     odd += w >> 16    (the high samples alone; one SDWA add)
// and at the end lo_total = mix - (odd << 16) (mod 2^32): exact while every
// total stays below 2^32, i.e. for up to 65537 channels.  Two channels' mix
// adds fuse into one v_add3, so two channel-words cost three instructions
// (0.75 VALU lane-operations per sample).  The float
// conversion rounds to nearest even above 2^24, as the host's int64-to-float
// conversion does.
//
// Grid order: blockIdx.x runs over DM blocks, so the workgroups resident at any
// time share a few time tiles and read the same input rows through L2/MALL.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_internal.h"
#include "tile_order.h"

namespace dd {
namespace {

constexpr uint32_t kOddSel = 0x0C030C01u;
constexpr int kBufferRsrcFlags = 0x00020000;  // raw (untyped) buffer access, word 3 of the descriptor

// Read-only tables read with wave-uniform addresses go through the constant
// address space, which the compiler always serves with scalar loads; a vector
// load here would make the wave wait for every global read in flight.
template <typename T>
__device__ __forceinline__ T scalar_load(const T *p, int64_t i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}  // v_perm: bytes 1 and 3 into bytes 0 and 2, zeros elsewhere

// Unpack 8 bytes of 4-bit samples (even sample in the low nibble) into 16 bytes.
__device__ __forceinline__ uint4 unpack_u4(uint2 p) {
  const uint32_t lo0 = p.x & 0x0F0F0F0Fu, hi0 = (p.x >> 4) & 0x0F0F0F0Fu;
  const uint32_t lo1 = p.y & 0x0F0F0F0Fu, hi1 = (p.y >> 4) & 0x0F0F0F0Fu;
  uint4 r;
  r.x = __builtin_amdgcn_perm(hi0, lo0, 0x05010400u);
  r.y = __builtin_amdgcn_perm(hi0, lo0, 0x07030602u);
  r.z = __builtin_amdgcn_perm(hi1, lo1, 0x05010400u);
  r.w = __builtin_amdgcn_perm(hi1, lo1, 0x07030602u);
  return r;
}

// acc + (w >> 16) as one SDWA add (the high half of w selected as the
// operand).  The compiler otherwise emits a shift per word and fuses two
// channels' shifted words into a v_add3: three instructions per two
// channel-words here against four.
__device__ __forceinline__ uint32_t add_high_half(uint32_t acc, uint32_t w) {
  uint32_t r;
  asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
      : "=v"(r)
      : "v"(acc), "v"(w));
  return r;
}

// Copies of a staged row: four byte phases for 8- and 4-bit samples, two
// (0 and 2 bytes) for 16-bit samples.
template <int BITS>
constexpr int num_phases() { return BITS == 16 ? 2 : 4; }

// Write the shifted copies of one 16-byte chunk whose phase-0 words are
// w[0..3] and whose next word is w[4]; `dst` points at the chunk in copy 0.
template <int BITS>
__device__ __forceinline__ void write_phases(uint8_t *dst, int row_bytes, const uint32_t (&w)[5]) {
#pragma unroll
  for (int p = 1; p < num_phases<BITS>(); ++p) {
    const int sh = BITS == 16 ? 2 * p : p;  // byte shift of copy p
    uint4 v;
    v.x = __builtin_amdgcn_alignbyte(w[1], w[0], sh);
    v.y = __builtin_amdgcn_alignbyte(w[2], w[1], sh);
    v.z = __builtin_amdgcn_alignbyte(w[3], w[2], sh);
    v.w = __builtin_amdgcn_alignbyte(w[4], w[3], sh);
    *(uint4 *)(dst + p * row_bytes) = v;
  }
}

template <int NS, int R>
__device__ __forceinline__ void flush(uint32_t (&mix)[R][NS / 4], uint32_t (&odd)[R][NS / 4], uint32_t (&tot)[R][NS]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int k = 0; k < NS / 4; ++k) {
      const uint32_t od = odd[r][k];
      const uint32_t ev = mix[r][k] - (od << 8);
      tot[r][4 * k + 0] += ev & 0xFFFFu;
      tot[r][4 * k + 1] += od & 0xFFFFu;
      tot[r][4 * k + 2] += ev >> 16;
      tot[r][4 * k + 3] += od >> 16;
      mix[r][k] = 0;
      odd[r][k] = 0;
    }
  }
}

// Epilogue of the 16-bit kernels for the two exact 32-bit totals of samples
// t and t + 1 (v0, v1), by OutMode: plain float32 conversion; the raw totals
// (the low-half plane of a split sum, kept in the output buffer); or the
// combination with those raw totals, low + 2^16 * this, converted once.  The
// combined sum is below 2^49, so its double is exact and the conversion to
// float rounds once, to nearest even, as the conversion of the exact sum would.
__device__ __forceinline__ float combine_split(uint32_t lo_total, uint32_t hi_total) {
  return (float)((double)lo_total + 65536.0 * (double)hi_total);
}

// The mode is a template parameter: a run-time choice here raised the 16-bit
// kernels' register use from 116 to 138 VGPRs, below two workgroups per CU.
template <int MODE>
__device__ __forceinline__ void store_u16_pair(float *orow, int64_t t, int64_t n_out, uint32_t v0, uint32_t v1) {
  if (t >= n_out) return;
  const bool both = t + 1 < n_out;
  if constexpr (MODE == kOutRawTotals) {
    if (both)
      *(uint2 *)(orow + t) = make_uint2(v0, v1);
    else
      *(uint32_t *)(orow + t) = v0;
  } else if constexpr (MODE == kOutCombineHigh) {
    if (both) {
      const uint2 lo = *(const uint2 *)(orow + t);
      *(float2 *)(orow + t) = make_float2(combine_split(lo.x, v0), combine_split(lo.y, v1));
    } else {
      orow[t] = combine_split(*(const uint32_t *)(orow + t), v0);
    }
  } else {
    if (both)
      *(float2 *)(orow + t) = make_float2((float)v0, (float)v1);
    else
      orow[t] = (float)v0;
  }
}

// Kernel arguments shared by the plain and the batched kernels.
struct IntArgs {
  const uint8_t *x;       // [n_chan][pitch] bytes
  const uint32_t *offs;   // [n_dblk][NW][n_chan][words]: LDS offsets (see build_int_tables, int_entry_words)
  const int32_t *sbase;   // [n_dblk][n_chan]: stage base (first-DM shift rounded down to the unit)
  float *out;             // [n_dm][out_pitch]
  int64_t pitch, n_samp, n_out, out_pitch;
  int32_t n_chan, n_dm, row_bytes;
};

// Workgroup barrier for LDS hand-offs.  __syncthreads() also waits for every
// outstanding global load (vmcnt(0)), which would stall on the staging reads
// kept in flight across blocks; only this wave's LDS operations must have
// completed before the barrier.  The asm is a compiler memory barrier too.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Staging.  Channel blocks stream through a ring of kRing LDS slots with
// direct global->LDS buffer loads (no registers involved), kRing-1 blocks
// ahead of the block being summed.  A slot holds the raw input bytes of the
// block's rows (packed nibbles for 4-bit input); from it the workgroup builds
// the four byte-phase copies the sum reads, one block ahead.  A block always
// has CB channels: channels past the last one are staged as zero rows.
//
// The loads of a block are cut in segments of 64 lanes x 16 bytes of one row;
// segment s goes to wave s % NW, so the channel and its staging base are
// wave-uniform (scalar loads).  Every wave issues exactly MAXT loads per block
// (out-of-range rows, segments and blocks read zeros into a scratch area), so
// a fixed s_waitcnt vmcnt count waits for exactly one block.
constexpr int kStageSegs = 16;  // host keeps CB * ceil(ring row bytes / 1024) <= kStageSegs
constexpr int kRing = 3;

typedef __attribute__((address_space(3))) void lds_void_t;
typedef int v4i_t __attribute__((ext_vector_type(4)));

// Raw buffer descriptor over [base, base + bytes): reads past the end return 0.
// The arguments are wave-uniform; readfirstlane keeps the descriptor in SGPRs
// (the inline-asm loads take it as an "s" operand) even where the compiler
// computed a part of it with vector instructions.
__device__ __forceinline__ v4i_t make_rsrc(const void *base, int bytes) {
  const uint64_t a = (uint64_t)base;
  v4i_t r;
  r.x = __builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  r.y = __builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));  // stride 0
  r.z = __builtin_amdgcn_readfirstlane(bytes);
  r.w = kBufferRsrcFlags;
  return r;
}

// 16 bytes per lane from buffer offset `voff` straight into LDS at
// lds_addr + 16 * lane.  Written as asm so that the compiler does not insert
// its own conservative wait for these LDS writes before every later LDS read:
// the kernel waits for them explicitly (wait_vmcnt) and orders them with
// lds_barrier().
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"  // m0 is reserved, but nothing else in these kernels uses it
__device__ __forceinline__ void dma16(const v4i_t &rs, uint32_t voff, uint32_t lds_addr) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tbuffer_load_dwordx4 %0, %2, 0 offen lds"
               :
               : "v"(voff), "s"(lds_addr), "s"(rs)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// LDS layout of a tile: two phase buffers, the ring, a 1 KB scratch area.
struct TileLds {
  int row_bytes;    // one copy of a row
  int phase_buf;    // CB * copies * row_bytes
  int ring_row;     // stride of a raw row in a ring slot (multiple of 16, >= raw bytes + 16)
  int ring_slot;    // CB * ring_row
  int ring_base;    // 2 * phase_buf
  int scratch;      // ring_base + kRing * ring_slot
};

template <int CB, int BITS>
__device__ __forceinline__ TileLds tile_lds(int row_bytes) {
  TileLds L;
  L.row_bytes = row_bytes;
  L.phase_buf = CB * num_phases<BITS>() * row_bytes;
  L.ring_row = (BITS == 4 ? row_bytes / 2 : row_bytes) + 16;
  L.ring_slot = CB * L.ring_row;
  L.ring_base = 2 * L.phase_buf;
  L.scratch = L.ring_base + kRing * L.ring_slot;
  return L;
}

// This wave's load segments of a block, the same for every block of a tile:
// segment s = wave + m*NW is 64 lanes x 16 bytes of channel cc starting at
// chunk j0 (segs = ceil(raw row bytes / 1 KiB) per channel).  Segments past
// the block's last are padding loads: every wave issues exactly MAXT loads per
// block, so a fixed vmcnt wait is exact; padding loads read nothing
// (zero-size buffer) and land in the scratch area.
template <int MAXT>
struct DmaPlan {
  int cc[MAXT];            // channel within the block (0 for padding)
  uint32_t lds_off[MAXT];  // byte offset of the segment inside a ring slot
  uint32_t voff[MAXT];     // this lane's byte offset inside the staged raw row
  bool ok[MAXT];           // a real segment (wave-uniform)
  bool lane_ok[MAXT];      // this lane's 16 bytes lie inside the raw row (always true for padding)
};

template <int NW, int CB, int MAXT, int BITS>
__device__ __forceinline__ DmaPlan<MAXT> dma_plan(const TileLds &L, int wave, int lane) {
  DmaPlan<MAXT> d;
  const int raw_bytes = BITS == 4 ? L.row_bytes / 2 : L.row_bytes;  // bytes of one row to stage
  const int segs = (raw_bytes + 1023) >> 10;
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const int s = wave + m * NW;
    d.ok[m] = s < CB * segs;
    const int cc = d.ok[m] ? s / segs : 0;
    const int j0 = d.ok[m] ? (s - cc * segs) << 6 : 0;  // first 16-byte chunk of the segment
    d.cc[m] = cc;
    d.lds_off[m] = (uint32_t)(cc * L.ring_row + 16 * j0);
    d.voff[m] = 16u * (uint32_t)(j0 + lane);
    d.lane_ok[m] = !d.ok[m] || 16 * (j0 + lane) < raw_bytes;
  }
  return d;
}

// Stage bases of the channels this wave loads for block `cb` (first channel).
// Scalar loads: issued one block before stage_dma needs them, so their
// latency hides behind a whole block of work.
template <int MAXT>
__device__ __forceinline__ void stage_bases(const IntArgs &a, const int32_t *sb, int cb, const DmaPlan<MAXT> &d,
                                            int32_t (&base)[MAXT]) {
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const int c = __builtin_amdgcn_readfirstlane(min(cb + d.cc[m], a.n_chan - 1));
    base[m] = scalar_load(sb, c);
  }
}

// Issue the direct loads of block `cb` (first channel) into ring slot `slot`;
// `base` comes from stage_bases for the same block.
template <int MAXT, int BITS>
__device__ __forceinline__ void stage_dma(const IntArgs &a, const DmaPlan<MAXT> &d, const int32_t (&base_in)[MAXT],
                                          int64_t t0, int cb, uint8_t *lds, const TileLds &L, int slot) {
  // Bounds are checked per 32-bit word, so the limit is the row length rounded
  // up to 16 bytes (still inside the row pitch).
  const int64_t row_len = BITS == 4 ? a.n_samp / 2 : BITS == 16 ? 2 * a.n_samp : a.n_samp;
  const int row_valid_bytes = (int)((row_len + 15) & ~(int64_t)15);
  const uint32_t slot_addr =
      __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)(lds + L.ring_base + slot * L.ring_slot));
  const uint32_t scratch_addr = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)(lds + L.scratch));
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const bool chan_ok = d.ok[m] && cb + d.cc[m] < a.n_chan;  // wave-uniform
    const int c = __builtin_amdgcn_readfirstlane(min(cb + d.cc[m], a.n_chan - 1));
    const int32_t base = chan_ok ? base_in[m] : 0;
    const v4i_t rs = make_rsrc(a.x + (int64_t)c * a.pitch, chan_ok ? row_valid_bytes : 0);
    // first staged byte of the row: sample t0 + base (a multiple of 16 bytes' worth of samples)
    const uint32_t row0 = BITS == 4    ? (uint32_t)((t0 + base) >> 1)
                          : BITS == 16 ? (uint32_t)(2 * (t0 + base))
                                       : (uint32_t)(t0 + base);
    const uint32_t lds_addr = d.ok[m] ? slot_addr + d.lds_off[m] : scratch_addr;
    if (d.lane_ok[m]) dma16(rs, row0 + d.voff[m], lds_addr);
  }
}

// This thread's chunks of a block: chunk i = threadIdx.x + NT*n is chunk j of
// row cc, i = cc * row_chunks + j.  The first (cc, j) and the per-step
// increments are computed once per tile; the walk needs no division.
struct ChunkWalk {
  int cc0, j0, dcc, dj, row_chunks;
};

template <int NT>
__device__ __forceinline__ ChunkWalk chunk_walk(const TileLds &L) {
  ChunkWalk w;
  w.row_chunks = L.row_bytes >> 4;
  w.cc0 = (int)threadIdx.x / w.row_chunks;
  w.j0 = (int)threadIdx.x - w.cc0 * w.row_chunks;
  w.dcc = NT / w.row_chunks;
  w.dj = NT - w.dcc * w.row_chunks;
  return w;
}

// Build the shifted copies of block (ring slot `slot`) into phase buffer `pb`.
template <int NT, int CB, int BITS>
__device__ __forceinline__ void build_phases(uint8_t *lds, const TileLds &L, const ChunkWalk &cw, int slot, int pb) {
  const uint8_t *ring = lds + L.ring_base + slot * L.ring_slot;
  uint8_t *dst = lds + pb * L.phase_buf;
  for (int cc = cw.cc0, j = cw.j0; cc < CB;) {
    uint32_t w[5];
    if (BITS != 4) {
      const uint8_t *src = ring + cc * L.ring_row + 16 * j;
      const uint4 v = *(const uint4 *)src;
      w[0] = v.x;
      w[1] = v.y;
      w[2] = v.z;
      w[3] = v.w;
      w[4] = *(const uint32_t *)(src + 16);  // past the row: only feeds samples beyond every window
    } else {
      const uint8_t *src = ring + cc * L.ring_row + 8 * j;
      const uint2 pv = *(const uint2 *)src;
      const uint4 v = unpack_u4(pv);
      const uint4 n = unpack_u4(make_uint2(*(const uint32_t *)(src + 8), 0u));
      w[0] = v.x;
      w[1] = v.y;
      w[2] = v.z;
      w[3] = v.w;
      w[4] = n.x;
    }
    uint8_t *p0 = dst + cc * num_phases<BITS>() * L.row_bytes + 16 * j;
    *(uint4 *)p0 = make_uint4(w[0], w[1], w[2], w[3]);
    write_phases<BITS>(p0, L.row_bytes, w);
    cc += cw.dcc;
    j += cw.dj;
    if (j >= cw.row_chunks) {
      j -= cw.row_chunks;
      ++cc;
    }
  }
}

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // s_waitcnt encoding on gfx9: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] << 14
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// One tile: DM block `dblk`, time tile `tblk`.  OM: the OutMode of the
// 16-bit epilogue (kOutFloat for other inputs).
template <int NS, int R, int NW, int CB, int BITS, int OM>
__device__ __forceinline__ void fwd_int_tile(uint8_t *lds, const IntArgs &a, int dblk, int tblk) {
  constexpr int NT = NW * 64;
  constexpr int NPH = num_phases<BITS>();
  constexpr int NWD = BITS == 16 ? NS / 2 : NS / 4;  // 32-bit words per lane and window
  constexpr int RP = R < 2 ? 2 : R;  // uint16 slots per channel in the offset table
  constexpr int NOW = RP / 2;        // uint32 words per channel
  constexpr int MAXT = (kStageSegs + NW - 1) / NW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)tblk * (64 * NS);
  const int chan_pad = (a.n_chan + CB - 1) / CB * CB;
  const uint32_t *woffs = a.offs + ((int64_t)dblk * NW + wave) * chan_pad * NOW;
  const int32_t *sb = a.sbase + (int64_t)dblk * a.n_chan;
  const TileLds L = tile_lds<CB, BITS>(a.row_bytes);

  // 8/4-bit: mix/odd are the SIMD-in-word accumulators, tot the flushed totals.
  // 16-bit: mix sums whole words, odd the high samples (see the file comment).
  uint32_t tot[R][NS], mix[R][NWD], odd[R][NWD];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int j = 0; j < NS; ++j) tot[r][j] = 0;
#pragma unroll
    for (int k = 0; k < NWD; ++k) mix[r][k] = odd[r][k] = 0;
  }

  const int nblk = chan_pad / CB;
  const DmaPlan<MAXT> dp = dma_plan<NW, CB, MAXT, BITS>(L, wave, lane);
  int32_t bases[MAXT];
#pragma unroll
  for (int k = 0; k < kRing; ++k) {
    stage_bases<MAXT>(a, sb, k * CB, dp, bases);
    stage_dma<MAXT, BITS>(a, dp, bases, t0, k * CB, lds, L, k);
  }
  stage_bases<MAXT>(a, sb, kRing * CB, dp, bases);
  // Offsets of block 0; each iteration fetches those of the next block.
  uint32_t ow[CB * NOW];
#pragma unroll
  for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, q);
  const ChunkWalk cw = chunk_walk<NT>(L);
  wait_vmcnt<(kRing - 1) * MAXT>();
  lds_barrier();
  build_phases<NT, CB, BITS>(lds, L, cw, 0, 0);

  const uint8_t *lane_base = lds + 4 * lane;
  int since_flush = 0;
  for (int b = 0; b < nblk; ++b) {
    // Block b+1's loads have landed (this wave's); after the barrier, every
    // wave's have, block b's phase copies are complete, and nobody reads ring
    // slot b % kRing or phase buffer (b+1) % 2 any more.
    wait_vmcnt<(kRing - 2) * MAXT>();
    lds_barrier();
    stage_dma<MAXT, BITS>(a, dp, bases, t0, (b + kRing) * CB, lds, L, b % kRing);  // zeros past the end
    if (b + 1 < nblk) build_phases<NT, CB, BITS>(lds, L, cw, (b + 1) % kRing, (b + 1) & 1);
    // Sum block b.  Each (channel, DM row) pair reads NS/4 aligned words of
    // the byte phase that puts its window on a word boundary; the table entry
    // is that word's byte offset inside the channel's four copies.  Lane i
    // owns words i, i+64, i+128, ... of the window, so every read is one
    // contiguous, bank-conflict-free 256-byte access per wave.  Reads run one
    // step ahead of the adds in a second register set, so every wave keeps LDS
    // reads in flight while it adds: for 8-bit data a channel pair ahead, with
    // the schedule pinned (the pair's reads, then the previous pair's adds;
    // measured 3% faster on 8192 channels), for 4- and 16-bit data one channel
    // ahead (the pinned pair schedule was 29% slower for 16-bit data).
    const uint8_t *blk = lane_base + (b & 1) * L.phase_buf;
    uint32_t wv[2][R][NWD];
    auto read_chan = [&](int cc, uint32_t (&dst)[R][NWD]) {
      const uint8_t *chan = blk + cc * NPH * L.row_bytes;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t e = (ow[cc * NOW + (r >> 1)] >> (16 * (r & 1))) & 0xFFFFu;
        const uint32_t *p = (const uint32_t *)(chan + e);
#pragma unroll
        for (int k = 0; k < NWD; ++k) dst[r][k] = p[64 * k];
      }
    };
    uint32_t wp[2][2][R][NWD];  // channel pairs: the pair after the one being summed is in flight
    if constexpr (BITS == 8 && CB >= 2) {
      read_chan(0, wp[0][0]);
      read_chan(1, wp[0][1]);
#pragma unroll
      for (int pc = 0; pc < CB / 2; ++pc) {
        if (2 * pc + 2 < CB) {
          read_chan(2 * pc + 2, wp[(pc + 1) & 1][0]);
          read_chan(2 * pc + 3, wp[(pc + 1) & 1][1]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NWD; ++k) {
              const uint32_t w = wp[pc & 1][h][r][k];
              if constexpr (BITS == 16) {
                mix[r][k] += w;
                odd[r][k] = add_high_half(odd[r][k], w);
              } else {
                mix[r][k] += w;
                odd[r][k] += __builtin_amdgcn_perm(w, w, kOddSel);
              }
            }
        if (2 * pc + 2 < CB) {
          // issue the next pair's reads first, then this pair's adds
          __builtin_amdgcn_sched_group_barrier(0x100, R * NWD, 0);      // DS reads: the next pair
          __builtin_amdgcn_sched_group_barrier(0x002, 8 * R * NWD, 0);  // VALU: this pair's adds
        }
      }
    } else {
      read_chan(0, wv[0]);
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        if (cc + 1 < CB) read_chan(cc + 1, wv[(cc + 1) & 1]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int k = 0; k < NWD; ++k) {
            const uint32_t w = wv[cc & 1][r][k];
            if constexpr (BITS == 16) {
              mix[r][k] += w;
              odd[r][k] = add_high_half(odd[r][k], w);
            } else {
              mix[r][k] += w;
              odd[r][k] += __builtin_amdgcn_perm(w, w, kOddSel);
            }
          }
        }
      }
    }
    if constexpr (BITS != 16) {
      since_flush += CB;
      if (since_flush >= 256 || b + 1 == nblk) {
        flush<NS, R>(mix, odd, tot);
        since_flush = 0;
      }
    }
    // Scalar loads for the next iteration: its offsets and the stage bases of
    // the block it stages.  Issued after this block's LDS reads, so that no
    // wait for them (LDS and scalar loads share one counter) falls inside the
    // summation; the barrier's wait absorbs their latency.
    const int oi = __builtin_amdgcn_readfirstlane(min(b + 1, nblk - 1) * CB * NOW);
#pragma unroll
    for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, oi + q);
    stage_bases<MAXT>(a, sb, (b + kRing + 1) * CB, dp, bases);
  }
  wait_vmcnt<0>();  // the trailing all-zero loads must land before the LDS is reused
  lds_barrier();

  // Word k of lane i holds samples t0 + 4*(i + 64k) + 0..3 (16-bit: t0 +
  // 2*(i + 64k) + 0..1): stores are contiguous across the wave.
  const int d0 = dblk * (NW * R) + wave * R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int d = d0 + r;
    if (d >= a.n_dm) break;
    float *orow = a.out + (int64_t)d * a.out_pitch;
    if constexpr (BITS == 16) {
#pragma unroll
      for (int k = 0; k < NWD; ++k) {
        const int64_t t = t0 + 2 * (int64_t)(lane + 64 * k);
        const uint32_t lo = mix[r][k] - (odd[r][k] << 16);
        store_u16_pair<OM>(orow, t, a.n_out, lo, odd[r][k]);
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < NS / 4; ++k) {
      const int64_t t = t0 + 4 * (int64_t)(lane + 64 * k);
      if (t + 3 < a.n_out) {
        *(float4 *)(orow + t) = make_float4((float)tot[r][4 * k], (float)tot[r][4 * k + 1], (float)tot[r][4 * k + 2],
                                            (float)tot[r][4 * k + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t + i < a.n_out) orow[t + i] = (float)tot[r][4 * k + i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 8-bit staging by phase loads.  The four byte-phase copies of a staged row are
// loaded straight from memory into LDS, copy p from byte p of the row on
// (16-byte loads at byte offsets that are not multiples of 4; the memory
// pipeline handles them).  Each (channel, block) gets a buffer descriptor
// based at its first staged byte whose record bound ends at the row length
// rounded up to 16 bytes (inside the row pitch), so nothing past the pitch is
// read.  The bound is checked per 32-bit word of a load: copy 0's words are
// aligned and all arrive, but in copies 1..3 the one word that straddles the
// bound reads as zero although its first 4 - p bytes lie inside it.  Where a
// staged row reaches that far (the last time tiles), the wave that loaded the
// word rebuilds it from copy 0's last word (a byte shift) before the block's
// barrier.  No phase-building pass, no raw ring: channel blocks stream through
// kPhaseRing slots of CB channels x 4 copies, kPhaseRing - 1 blocks ahead of
// the summation, with one barrier per block.  The table entry of a (channel, DM
// row) is the byte offset of its window's first word from the start of the
// slot (padding channels past the last: their own zero row), so the summation
// needs one address add per (channel, row).  16-bit rows take two copies, from
// bytes 0 and 2 (every 16-bit window then starts on a word of one of them),
// with the same straddling-word rebuild for copy 1.
//
// Loads per block: each of the CB * SEGS (channel, 1 KiB segment) pairs issues
// its phase loads (four; two for 16-bit rows) from one wave; pair j goes to
// wave j % NW, so every wave issues exactly the same number of loads per block
// (padding loads of zero bytes into a sink keep the count fixed) and one vmcnt
// wait is exact.
constexpr int kPhaseRing = 3;

template <int CB, int SEGS, int NW>
constexpr int phase_pairs_per_wave() { return (CB * SEGS + NW - 1) / NW; }

// Copies of a staged row in the phase-load forms: the four byte phases for
// 8-bit samples; for packed 4-bit samples the eight nibble phases, of which
// the byte phases are the even ones (copy 2p = byte phase p); for 16-bit
// samples two, from bytes 0 and 2.
template <int BITS>
constexpr int phase_copies() { return BITS == 4 ? 8 : BITS == 16 ? 2 : 4; }

// Loads per (channel, segment) pair and their byte step: the copies that come
// straight from memory (all of them but the odd nibble phases).
template <int BITS>
constexpr int phase_loads() { return BITS == 16 ? 2 : 4; }
template <int BITS>
constexpr int phase_load_step() { return BITS == 16 ? 2 : 1; }

// Bytes of row from sample s on (4-bit rows hold two samples per byte; every
// staged row starts on a multiple of 32 samples).
template <int BITS>
__device__ __forceinline__ int64_t phase_bytes(int64_t s) { return BITS == 4 ? s >> 1 : BITS == 16 ? 2 * s : s; }

// This wave's (channel, segment) pairs: channel within the block, segment.
template <int CB, int SEGS, int NW>
struct PhasePlan {
  static constexpr int J = phase_pairs_per_wave<CB, SEGS, NW>();
  int cc[J];           // channel within the block (0 for padding)
  bool ok[J];          // a real pair (wave-uniform)
  uint32_t lds_off[J];  // LDS byte offset of the pair's copy 0 segment inside a slot
  uint32_t voff[J];    // this lane's byte offset in the staged row, copy 0
  int seg0[J];         // first byte of the pair's segment in the staged row
  bool lane_ok[J];     // this lane's 16 bytes lie inside the copy (true for padding)
};

template <int CB, int SEGS, int NW, int BITS>
__device__ __forceinline__ PhasePlan<CB, SEGS, NW> phase_plan(int row_bytes, int wave, int lane) {
  PhasePlan<CB, SEGS, NW> d;
#pragma unroll
  for (int m = 0; m < PhasePlan<CB, SEGS, NW>::J; ++m) {
    const int j = wave + m * NW;
    const int cc = j / SEGS, seg = j - cc * SEGS;
    d.ok[m] = j < CB * SEGS && 1024 * seg < row_bytes;
    d.cc[m] = d.ok[m] ? cc : 0;
    d.lds_off[m] = d.ok[m] ? (uint32_t)(cc * phase_copies<BITS>() * row_bytes + 1024 * seg) : 0u;
    d.voff[m] = (uint32_t)(1024 * seg + 16 * lane);
    d.seg0[m] = 1024 * seg;
    d.lane_ok[m] = !d.ok[m] || 1024 * seg + 16 * lane < row_bytes;
  }
  return d;
}

// Issue this wave's phase loads of block `cb` (first channel) into ring slot
// `slot`; `base` holds the stage bases of the wave's channels for that block.
// Byte phase p goes to copy p (8-bit) or copy 2p (4-bit); 16-bit rows load
// copies 0 and 1 from bytes 0 and 2.
template <int CB, int SEGS, int NW, int BITS>
__device__ __forceinline__ void phase_dma(const IntArgs &a, const PhasePlan<CB, SEGS, NW> &d,
                                          const int32_t (&base_in)[PhasePlan<CB, SEGS, NW>::J], int64_t t0, int cb,
                                          uint8_t *lds, int slot_bytes, int slot, uint32_t sink_addr) {
  const uint32_t slot_addr =
      __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)(lds + slot * slot_bytes));
  const int64_t bound = (phase_bytes<BITS>(a.n_samp) + 15) & ~(int64_t)15;  // row bytes rounded up to 16 (<= pitch)
#pragma unroll
  for (int m = 0; m < PhasePlan<CB, SEGS, NW>::J; ++m) {
    const bool chan_ok = d.ok[m] && cb + d.cc[m] < a.n_chan;  // wave-uniform
    const int c = __builtin_amdgcn_readfirstlane(min(cb + d.cc[m], a.n_chan - 1));
    // first staged byte of the row (a multiple of 16) and the bytes from there to the bound
    const int64_t row0 = chan_ok ? phase_bytes<BITS>(t0 + base_in[m]) : 0;
    const int64_t left = bound - row0;
    const int bytes = chan_ok && left > 0 ? (int)min(left, (int64_t)0x7fffffff) : 0;
    const v4i_t rs = make_rsrc(a.x + (int64_t)c * a.pitch + row0, bytes);
    const uint32_t dst = d.ok[m] ? slot_addr + d.lds_off[m] : sink_addr;
    // padding: all of them into the sink
    constexpr int NL = phase_loads<BITS>();
    const uint32_t copy_step = d.ok[m] ? (uint32_t)(phase_copies<BITS>() / NL * a.row_bytes) : 0u;
    if (d.lane_ok[m]) {
#pragma unroll
      for (int ph = 0; ph < NL; ++ph) dma16(rs, d.voff[m] + ph * phase_load_step<BITS>(), dst + ph * copy_step);
    }
  }
}

// Stage bases of this wave's channels of block `cb` (scalar loads, one block early).
template <int CB, int SEGS, int NW>
__device__ __forceinline__ void phase_bases(const IntArgs &a, const int32_t *sb, int cb,
                                            const PhasePlan<CB, SEGS, NW> &d,
                                            int32_t (&base)[PhasePlan<CB, SEGS, NW>::J]) {
#pragma unroll
  for (int m = 0; m < PhasePlan<CB, SEGS, NW>::J; ++m) {
    const int c = __builtin_amdgcn_readfirstlane(min(cb + d.cc[m], a.n_chan - 1));
    base[m] = scalar_load(sb, c);
  }
}

// Rebuild, in the loaded copies 1.. of this wave's channels of block `cb`
// (ring slot `slot`), the word that straddles the load bound (see above).  The
// copy loaded from byte o holds at copy position k = bound - 4 the row bytes
// k + o .. k + o + 3, of which those below the bound are copy 0's word at k
// shifted down by o bytes; the rest lie past the row and feed no output.  Call
// after this wave's loads of the block have landed and before the block's
// barrier.
template <int CB, int SEGS, int NW, int BITS>
__device__ __forceinline__ void phase_fix_tail(const IntArgs &a, const PhasePlan<CB, SEGS, NW> &d, const int32_t *sb,
                                               int64_t t0, int cb, uint8_t *lds, int slot_bytes, int slot, int lane) {
  const int64_t bound = (phase_bytes<BITS>(a.n_samp) + 15) & ~(int64_t)15;
  constexpr int NL = phase_loads<BITS>();
  const int step = phase_copies<BITS>() / NL * a.row_bytes;  // load p's copy is at p * step
#pragma unroll
  for (int m = 0; m < PhasePlan<CB, SEGS, NW>::J; ++m) {
    const int c = cb + d.cc[m];
    if (!d.ok[m] || c >= a.n_chan) continue;  // wave-uniform
    const int64_t k = bound - phase_bytes<BITS>(t0 + scalar_load(sb, c)) - 4;
    if (k < d.seg0[m] || k >= d.seg0[m] + 1024 || k >= a.row_bytes) continue;  // not in this wave's segment
    if (lane < NL - 1) {
      uint8_t *row = lds + slot * slot_bytes + d.cc[m] * phase_copies<BITS>() * a.row_bytes + k;
      const uint32_t w0 = *(const uint32_t *)row;
      *(uint32_t *)(row + (lane + 1) * step) = w0 >> (8 * phase_load_step<BITS>() * (lane + 1));
    }
  }
}

// Does any staged row of tile t0 reach the word that straddles the load bound?
// (Stage bases are at most the largest shift, n_samp - n_out.)
template <int BITS>
__device__ __forceinline__ bool phase_near_end(const IntArgs &a, int64_t t0) {
  const int64_t bound = (phase_bytes<BITS>(a.n_samp) + 15) & ~(int64_t)15;
  return phase_bytes<BITS>(t0 + (a.n_samp - a.n_out)) + a.row_bytes + 4 > bound;
}

// Phase-load tile for 8-bit and 16-bit input.  8-bit: the four byte-phase
// copies, SIMD-in-word mix/odd sums flushed every 256 channels, channel pairs
// read one pair ahead.  16-bit: the copies from bytes 0 and 2, mix/odd sums of
// whole words and their high halves (exact 32-bit totals, no flush), one
// channel read ahead; the epilogue by OutMode as in the ring form.
template <int NS, int R, int NW, int CB, int SEGS, int BITS, int OM>
__device__ __forceinline__ void fwd_byte_phase_tile(uint8_t *lds, const IntArgs &a, int dblk, int tblk) {
  static_assert(BITS == 8 || BITS == 16, "byte-phase tiles take 8- or 16-bit samples");
  constexpr int NWD = BITS == 16 ? NS / 2 : NS / 4;  // 32-bit words per lane and window
  constexpr int NOW = R;  // one 32-bit table entry per (channel, row)
  constexpr int J = PhasePlan<CB, SEGS, NW>::J;
  constexpr int LOADS = phase_loads<BITS>() * J;  // loads per wave and block
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)tblk * (64 * NS);
  const int chan_pad = (a.n_chan + CB - 1) / CB * CB;
  const uint32_t *woffs = a.offs + ((int64_t)dblk * NW + wave) * chan_pad * NOW;
  const int32_t *sb = a.sbase + (int64_t)dblk * a.n_chan;
  const int slot_bytes = CB * phase_copies<BITS>() * a.row_bytes;
  const uint32_t sink_addr =
      __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)(lds + kPhaseRing * slot_bytes));

  // 8-bit: mix/odd are the SIMD-in-word accumulators, tot the flushed totals.
  // 16-bit: mix sums whole words, odd their high halves; no tot.
  uint32_t tot[R][BITS == 16 ? 1 : NS], mix[R][NWD], odd[R][NWD];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if constexpr (BITS != 16) {
#pragma unroll
      for (int j = 0; j < NS; ++j) tot[r][j] = 0;
    }
#pragma unroll
    for (int k = 0; k < NWD; ++k) mix[r][k] = odd[r][k] = 0;
  }

  const int nblk = chan_pad / CB;
  const PhasePlan<CB, SEGS, NW> dp = phase_plan<CB, SEGS, NW, BITS>(a.row_bytes, wave, lane);
  int32_t bases[J];
#pragma unroll
  for (int k = 0; k < kPhaseRing - 1; ++k) {
    phase_bases<CB, SEGS, NW>(a, sb, k * CB, dp, bases);
    phase_dma<CB, SEGS, NW, BITS>(a, dp, bases, t0, k * CB, lds, slot_bytes, k, sink_addr);
  }
  phase_bases<CB, SEGS, NW>(a, sb, (kPhaseRing - 1) * CB, dp, bases);
  uint32_t ow[CB * NOW];
#pragma unroll
  for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, q);

  const uint8_t *lane_base = lds + 4 * lane;
  const bool near_end = phase_near_end<BITS>(a, t0);  // wave-uniform
  int since_flush = 0;
  for (int b = 0; b < nblk; ++b) {
    // This wave's loads of block b have landed; after the barrier every
    // wave's have, and no wave reads the slot of block b - 1 any more, which
    // the loads of block b + kPhaseRing - 1 then fill.
    wait_vmcnt<(kPhaseRing - 2) * LOADS>();
    if (near_end) phase_fix_tail<CB, SEGS, NW, BITS>(a, dp, sb, t0, b * CB, lds, slot_bytes, b % kPhaseRing, lane);
    lds_barrier();
    phase_dma<CB, SEGS, NW, BITS>(a, dp, bases, t0, (b + kPhaseRing - 1) * CB, lds, slot_bytes,
                                  (b + kPhaseRing - 1) % kPhaseRing, sink_addr);  // zeros past the last channel
    const uint8_t *blk = lane_base + (b % kPhaseRing) * slot_bytes;
    // The table entry is the window's byte offset from the slot start; lane i
    // owns words i, i+64, ... of the window (conflict-free ds_read2st64).
    auto read_chan = [&](int cc, uint32_t (&dst)[R][NWD]) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t e = ow[cc * NOW + r];
        const uint32_t *p = (const uint32_t *)(blk + e);
#pragma unroll
        for (int k = 0; k < NWD; ++k) dst[r][k] = p[64 * k];
      }
    };
    if constexpr (BITS == 16) {
      // one channel read ahead (a pair ahead would not fit the registers of 8 words per row)
      uint32_t wv[2][R][NWD];
      read_chan(0, wv[0]);
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        if (cc + 1 < CB) read_chan(cc + 1, wv[(cc + 1) & 1]);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k = 0; k < NWD; ++k) {
            const uint32_t w = wv[cc & 1][r][k];
            mix[r][k] += w;
            odd[r][k] = add_high_half(odd[r][k], w);
          }
      }
    } else {
      uint32_t wp[2][2][R][NWD];  // channel pairs: the pair after the one being summed is in flight
      read_chan(0, wp[0][0]);
      read_chan(1, wp[0][1]);
#pragma unroll
      for (int pc = 0; pc < CB / 2; ++pc) {
        if (2 * pc + 2 < CB) {
          read_chan(2 * pc + 2, wp[(pc + 1) & 1][0]);
          read_chan(2 * pc + 3, wp[(pc + 1) & 1][1]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NWD; ++k) {
              const uint32_t w = wp[pc & 1][h][r][k];
              mix[r][k] += w;
              odd[r][k] += __builtin_amdgcn_perm(w, w, kOddSel);
            }
        if (NWD > 2 && 2 * pc + 2 < CB) {  // pinned for wider windows; 8-sample windows run 1.4% faster unpinned
          __builtin_amdgcn_sched_group_barrier(0x100, R * NWD, 0);      // DS reads: the next pair
          __builtin_amdgcn_sched_group_barrier(0x002, 8 * R * NWD, 0);  // VALU: this pair's adds
        }
      }
      since_flush += CB;
      if (since_flush >= 256 || b + 1 == nblk) {
        flush<NS, R>(mix, odd, tot);
        since_flush = 0;
      }
    }
    const int oi = __builtin_amdgcn_readfirstlane(min(b + 1, nblk - 1) * CB * NOW);
#pragma unroll
    for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, oi + q);
    phase_bases<CB, SEGS, NW>(a, sb, (b + kPhaseRing) * CB, dp, bases);
  }
  wait_vmcnt<0>();  // the trailing loads must land before the LDS is reused
  lds_barrier();

  // Word k of lane i holds samples t0 + 4*(i + 64k) + 0..3 (16-bit: t0 +
  // 2*(i + 64k) + 0..1): stores are contiguous across the wave.
  const int d0 = dblk * (NW * R) + wave * R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int d = d0 + r;
    if (d >= a.n_dm) break;
    float *orow = a.out + (int64_t)d * a.out_pitch;
    if constexpr (BITS == 16) {
#pragma unroll
      for (int k = 0; k < NWD; ++k) {
        const int64_t t = t0 + 2 * (int64_t)(lane + 64 * k);
        const uint32_t lo = mix[r][k] - (odd[r][k] << 16);
        store_u16_pair<OM>(orow, t, a.n_out, lo, odd[r][k]);
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < NS / 4; ++k) {
      const int64_t t = t0 + 4 * (int64_t)(lane + 64 * k);
      if (t + 3 < a.n_out) {
        *(float4 *)(orow + t) = make_float4((float)tot[r][4 * k], (float)tot[r][4 * k + 1], (float)tot[r][4 * k + 2],
                                            (float)tot[r][4 * k + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t + i < a.n_out) orow[t + i] = (float)tot[r][4 * k + i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Packed 4-bit staging by phase loads.  A staged row stays packed (two samples
// per byte) in eight nibble-phase copies: copy q holds the row from nibble q
// on, so every window starts on a whole 32-bit word of the copy of its phase
// (v mod 8 for a window at nibble v).  The even copies are the byte phases and
// are loaded straight into LDS as in the 8-bit form (copy 2p from byte p; the
// word straddling the load bound is rebuilt the same way); the odd copies are
// built in LDS one block ahead of the summation: word k of copy 2p + 1 is words
// k and k + 1 of copy 2p funnel-shifted by one nibble.  LDS holds 4 bytes per
// staged sample, as the unpacked byte-phase form does, but the summation reads
// half the bytes (8 samples per word) and needs fewer instructions per sample:
//
// Exact SIMD-within-a-word sums of nibbles.  Per word w (nibbles n0..n7, n0 the
// earliest sample) a lane adds
//     E += w & 0x0F0F0F0F      (the even nibbles, one per byte lane)
//     S += w >> 4
// and two channels' words fuse into one v_add3 each: six instructions per 16
// samples.  w >> 4 is the odd nibbles in the byte lanes plus 16 times the even
// nibbles moved down one byte, so with no byte lane of E above 255 (at most 17
// channels) the odd-nibble sums are O = S - 16 * (E >> 8), S stays below 2^32.
// Every 16 channels the byte lanes of E and O are added into per-sample
// 32-bit totals with SDWA byte-select adds (eight per word).
//
// Block schedule: at iteration b this wave waits for its loads of block b + 1,
// the workgroup meets at the block barrier (block b + 1's even copies have all
// landed, block b's odd copies are complete, block b - 1's slot is free), the
// loads of block b + 2 go out, block b + 1's odd copies are built and block b
// is summed.  Three slots: the summation slot, the one being built, the one
// being loaded.

// acc + byte M of w (zero-extended): one SDWA add.
template <int M>
__device__ __forceinline__ uint32_t add_byte(uint32_t acc, uint32_t w) {
  uint32_t r;
  if constexpr (M == 0)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r) : "v"(acc), "v"(w));
  else if constexpr (M == 1)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
        : "=v"(r) : "v"(acc), "v"(w));
  else if constexpr (M == 2)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
        : "=v"(r) : "v"(acc), "v"(w));
  else
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
        : "=v"(r) : "v"(acc), "v"(w));
  return r;
}

// Flush the nibble sums of R rows x NWD words into the per-sample totals
// (sample 8k + j of the lane's word k at tot[r][8k + j]) and clear them.
template <int NWD, int R>
__device__ __forceinline__ void flush_u4(uint32_t (&ev)[R][NWD], uint32_t (&sh)[R][NWD], uint32_t (&tot)[R][8 * NWD]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int k = 0; k < NWD; ++k) {
      const uint32_t e = ev[r][k];
      const uint32_t o = sh[r][k] - ((e >> 4) & 0x0FFFFFF0u);  // S - 16 * (E >> 8)
      uint32_t *t = tot[r] + 8 * k;
      t[0] = add_byte<0>(t[0], e);
      t[2] = add_byte<1>(t[2], e);
      t[4] = add_byte<2>(t[4], e);
      t[6] = add_byte<3>(t[6], e);
      t[1] = add_byte<0>(t[1], o);
      t[3] = add_byte<1>(t[3], o);
      t[5] = add_byte<2>(t[5], o);
      t[7] = add_byte<3>(t[7], o);
      ev[r][k] = 0;
      sh[r][k] = 0;
    }
  }
}

// The odd-copy build's work split: the 16-byte chunks of a slot's even copies,
// numbered (channel, byte phase, chunk) and dealt round-robin over the
// workgroup's threads.  A thread's chunks sit at the same offsets from the
// slot start in every block, so they are worked out once per tile (rows of at
// most SEGS KiB give each thread at most N of them).
template <int CB, int SEGS, int NW>
struct OddPlan {
  static constexpr int N = (CB * 4 * SEGS * 64 + NW * 64 - 1) / (NW * 64);
  uint32_t off[N];  // byte offset of the chunk (in copy 2p) from the slot start; 0 past n
  int n;            // chunks of this thread
};

template <int CB, int SEGS, int NW>
__device__ __forceinline__ OddPlan<CB, SEGS, NW> odd_plan(int row_bytes) {
  constexpr int NT = NW * 64;
  OddPlan<CB, SEGS, NW> o;
  const int chunks = row_bytes >> 4;
  const int total = CB * 4 * chunks;
  const int tid = (int)threadIdx.x;
  o.n = tid < total ? (total - 1 - tid) / NT + 1 : 0;
#pragma unroll
  for (int m = 0; m < OddPlan<CB, SEGS, NW>::N; ++m) {
    const int i = tid + m * NT;
    const int cp = i / chunks, j = i - cp * chunks;  // cp = channel * 4 + byte phase
    o.off[m] = m < o.n ? (uint32_t)(2 * cp * row_bytes + 16 * j) : 0u;
  }
  return o;
}

// Build the odd nibble-phase copies of the CB channels of ring slot `slot`
// from the even ones: word k of copy 2p + 1 is words k and k + 1 of copy 2p
// shifted down by one nibble.  The last word of an odd copy takes its upper
// nibble from whatever follows copy 2p's row (the odd copy's first word, being
// written meanwhile): no window reads that word (rows carry a spare word).
template <int CB, int SEGS, int NW>
__device__ __forceinline__ void build_odd_nibbles(uint8_t *lds, int slot_bytes, int slot, int row_bytes,
                                                  const OddPlan<CB, SEGS, NW> &op) {
  constexpr int N = OddPlan<CB, SEGS, NW>::N;
  uint8_t *base = lds + slot * slot_bytes;
  // all reads first (chunks past this thread's count read chunk 0 and are not written back)
  uint4 v[N];
  uint32_t nx[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const uint8_t *src = base + op.off[m];
    v[m] = *(const uint4 *)src;
    nx[m] = *(const uint32_t *)(src + 16);
  }
#pragma unroll
  for (int m = 0; m < N; ++m) {
    uint4 o;
    o.x = __builtin_amdgcn_alignbit(v[m].y, v[m].x, 4);
    o.y = __builtin_amdgcn_alignbit(v[m].z, v[m].y, 4);
    o.z = __builtin_amdgcn_alignbit(v[m].w, v[m].z, 4);
    o.w = __builtin_amdgcn_alignbit(nx[m], v[m].w, 4);
    if (m < op.n) *(uint4 *)(base + op.off[m] + row_bytes) = o;  // copy 2p + 1
  }
}

template <int NS, int R, int NW, int CB, int SEGS>
__device__ __forceinline__ void fwd_u4_phase_tile(uint8_t *lds, const IntArgs &a, int dblk, int tblk) {
  static_assert(NS % 8 == 0, "4-bit phase tiles take whole 8-sample words per lane");
  constexpr int NWD = NS / 8;
  constexpr int NOW = R;  // one 32-bit table entry per (channel, row)
  constexpr int J = PhasePlan<CB, SEGS, NW>::J;
  constexpr int LOADS = 4 * J;  // loads per wave and block
  constexpr int kFlushChans = 16;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)tblk * (64 * NS);
  const int chan_pad = (a.n_chan + CB - 1) / CB * CB;
  const uint32_t *woffs = a.offs + ((int64_t)dblk * NW + wave) * chan_pad * NOW;
  const int32_t *sb = a.sbase + (int64_t)dblk * a.n_chan;
  const int slot_bytes = CB * 8 * a.row_bytes;
  const uint32_t sink_addr =
      __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)(lds + kPhaseRing * slot_bytes));

  uint32_t tot[R][NS], ev[R][NWD], sh[R][NWD];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int j = 0; j < NS; ++j) tot[r][j] = 0;
#pragma unroll
    for (int k = 0; k < NWD; ++k) ev[r][k] = sh[r][k] = 0;
  }

  const int nblk = chan_pad / CB;
  const PhasePlan<CB, SEGS, NW> dp = phase_plan<CB, SEGS, NW, 4>(a.row_bytes, wave, lane);
  const OddPlan<CB, SEGS, NW> op = odd_plan<CB, SEGS, NW>(a.row_bytes);
  const bool near_end = phase_near_end<4>(a, t0);  // wave-uniform
  int32_t bases[J];
  // Prologue: blocks 0 and 1 in flight; block 0's odd copies built.
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    phase_bases<CB, SEGS, NW>(a, sb, k * CB, dp, bases);
    phase_dma<CB, SEGS, NW, 4>(a, dp, bases, t0, k * CB, lds, slot_bytes, k, sink_addr);
  }
  phase_bases<CB, SEGS, NW>(a, sb, 2 * CB, dp, bases);
  uint32_t ow[CB * NOW];
#pragma unroll
  for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, q);
  wait_vmcnt<LOADS>();
  if (near_end) phase_fix_tail<CB, SEGS, NW, 4>(a, dp, sb, t0, 0, lds, slot_bytes, 0, lane);
  lds_barrier();
  build_odd_nibbles<CB, SEGS, NW>(lds, slot_bytes, 0, a.row_bytes, op);

  const uint8_t *lane_base = lds + 4 * lane;
  int since_flush = 0;
  for (int b = 0; b < nblk; ++b) {
    wait_vmcnt<0>();  // this wave's loads of block b + 1
    if (near_end) phase_fix_tail<CB, SEGS, NW, 4>(a, dp, sb, t0, (b + 1) * CB, lds, slot_bytes, (b + 1) % kPhaseRing, lane);
    lds_barrier();
    phase_dma<CB, SEGS, NW, 4>(a, dp, bases, t0, (b + 2) * CB, lds, slot_bytes, (b + 2) % kPhaseRing,
                               sink_addr);  // zeros past the last channel
    if (b + 1 < nblk) build_odd_nibbles<CB, SEGS, NW>(lds, slot_bytes, (b + 1) % kPhaseRing, a.row_bytes, op);
    const uint8_t *blk = lane_base + (b % kPhaseRing) * slot_bytes;
    auto read_chan = [&](int cc, uint32_t (&dst)[R][NWD]) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t e = ow[cc * NOW + r];
        const uint32_t *p = (const uint32_t *)(blk + e);
#pragma unroll
        for (int k = 0; k < NWD; ++k) dst[r][k] = p[64 * k];
      }
    };
    uint32_t wp[2][2][R][NWD];  // channel pairs: the pair after the one being summed is in flight
    read_chan(0, wp[0][0]);
    read_chan(1, wp[0][1]);
#pragma unroll
    for (int pc = 0; pc < CB / 2; ++pc) {
      if (2 * pc + 2 < CB) {
        read_chan(2 * pc + 2, wp[(pc + 1) & 1][0]);
        read_chan(2 * pc + 3, wp[(pc + 1) & 1][1]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < NWD; ++k) {
          const uint32_t w1 = wp[pc & 1][0][r][k], w2 = wp[pc & 1][1][r][k];
          ev[r][k] += (w1 & 0x0F0F0F0Fu) + (w2 & 0x0F0F0F0Fu);
          sh[r][k] += (w1 >> 4) + (w2 >> 4);
        }
    }
    since_flush += CB;
    if (since_flush + CB > kFlushChans || b + 1 == nblk) {
      flush_u4<NWD, R>(ev, sh, tot);
      since_flush = 0;
    }
    const int oi = __builtin_amdgcn_readfirstlane(min(b + 1, nblk - 1) * CB * NOW);
#pragma unroll
    for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, oi + q);
    phase_bases<CB, SEGS, NW>(a, sb, (b + 3) * CB, dp, bases);
  }
  wait_vmcnt<0>();  // the trailing loads must land before the LDS is reused
  lds_barrier();

  // Word k of lane i holds samples t0 + 8 * (i + 64k) + 0..7.
  const int d0 = dblk * (NW * R) + wave * R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int d = d0 + r;
    if (d >= a.n_dm) break;
    float *orow = a.out + (int64_t)d * a.out_pitch;
#pragma unroll
    for (int k = 0; k < NWD; ++k) {
      const int64_t t = t0 + 8 * (int64_t)(lane + 64 * k);
      const uint32_t *v = tot[r] + 8 * k;
      if (t + 7 < a.n_out) {
        *(float4 *)(orow + t) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
        *(float4 *)(orow + t + 4) = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (t + i < a.n_out) orow[t + i] = (float)v[i];
      }
    }
  }
}

// One tile of either staging form: SEGS == 0 is the ring form (fwd_int_tile),
// SEGS > 0 the phase-load form for 8-bit or packed 4-bit input with at most
// SEGS 1 KiB load segments per copy row.
template <int NS, int R, int NW, int CB, int SEGS, int BITS, int OM = kOutFloat>
__device__ __forceinline__ void int_tile(uint8_t *lds, const IntArgs &a, int dblk, int tblk) {
  if constexpr (SEGS == 0)
    fwd_int_tile<NS, R, NW, CB, BITS, OM>(lds, a, dblk, tblk);
  else if constexpr (BITS == 4)
    fwd_u4_phase_tile<NS, R, NW, CB, SEGS>(lds, a, dblk, tblk);
  else
    fwd_byte_phase_tile<NS, R, NW, CB, SEGS, BITS, OM>(lds, a, dblk, tblk);
}

// Waves per SIMD the compiler must leave room for: 8-wave shapes with at most
// 32 accumulated samples per lane are held to 128 VGPRs, so that two of their
// workgroups share a CU (4 waves per SIMD) when their LDS fits twice; wider
// shapes get no such limit (it would make them spill).
template <int NS, int R, int NW>
constexpr int min_waves_per_simd() { return NW == 8 && NS * R <= 32 ? 4 : 1; }

// One workgroup per tile; 1-D grid of n_dblk * n_tiles workgroups.
template <int NS, int R, int NW, int CB, int SEGS, int BITS, int OM = kOutFloat>
__global__ __launch_bounds__(NW * 64, (min_waves_per_simd<NS, R, NW>())) void fwd_int_kernel(IntArgs a, int n_dblk, int n_tiles, int order) {
  extern __shared__ __align__(16) uint8_t lds[];
  int dblk, tblk;
  tile_of(blockIdx.x, n_dblk, n_tiles, order, dblk, tblk);
  int_tile<NS, R, NW, CB, SEGS, BITS, OM>(lds, a, dblk, tblk);
}

__global__ void reset_counter_kernel(unsigned long long *counter) { *counter = 0ull; }

// Persistent batched forward kernel.  Workgroups claim work items (beam, DM
// block, time tile) from a device counter; items are numbered beam by beam
// with the beams in decreasing cost order and, inside a beam, DM block
// fastest: the items claimed at about the same time stage the same input rows
// (one time tile), which the XCDs' L2 caches then share, as in the XCD-aware
// orders of the plain launch (time tile fastest measured 2.3% slower than plain
// launches on the 48-beam job).  The claim of the next item
// is issued when an item starts and read when it ends, so its latency hides
// behind the tile.  Claims only grow, so the beam index only moves forward.
// A workgroup returns at its first claim past the last item: every wave
// reaches the exit.  Between items no extra barrier is needed for the LDS: a
// tile ends with all of its LDS reads complete behind its final barrier.
template <int NS, int R, int NW, int CB, int SEGS, int BITS>
__global__ __launch_bounds__(NW * 64, (min_waves_per_simd<NS, R, NW>())) void fwd_int_batched_kernel(const BeamDesc *__restrict__ beams, int n_beams,
                                                                   long long n_items,
                                                                   unsigned long long *__restrict__ counter) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ long long claimed;
  if (threadIdx.x == 0) claimed = (long long)atomicAdd(counter, 1ull);
  __syncthreads();
  long long item = claimed;
  int lo = 0;
  for (;;) {
    item = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)item >> 32))
                        << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)item));
    if (item >= n_items) return;
    unsigned long long next = 0;
    if (threadIdx.x == 0) next = atomicAdd(counter, 1ull);  // the following claim, read after this tile
    while (lo + 1 < n_beams && scalar_load(&beams[lo + 1].item_begin, 0) <= item) ++lo;
    const BeamDesc &b = beams[lo];
    const long long k = item - b.item_begin;
    const int tblk = (int)(k / b.tiles_d), dblk = (int)(k - (long long)tblk * b.tiles_d);
    IntArgs a;
    a.x = b.x;
    a.offs = b.offs;
    a.sbase = b.sbase;
    a.out = b.out;
    a.pitch = b.pitch;
    a.n_samp = b.n_samp;
    a.n_out = b.n_out;
    a.out_pitch = b.out_pitch;
    a.n_chan = b.n_chan;
    a.n_dm = b.n_dm;
    a.row_bytes = b.row_bytes;

    int_tile<NS, R, NW, CB, SEGS, BITS>(lds, a, dblk, tblk);
    if (threadIdx.x == 0) claimed = (long long)next;
    lds_barrier();  // publishes the claim; the tile's stores may still be in flight
    item = claimed;  // read before this wave's first barrier of the next tile; rewritten only after it
  }
}

// Compiled tile shapes (samples per lane, DM rows per wave, waves, channels
// per LDS stage, staging form: 0 = raw ring + phase build, any input; S > 0 =
// phase loads, copy rows of at most S KiB), in the order the plan tries them.
#define DD_INT_SHAPES(X)                                                                                    \
  X(16, 2, 16, 8, 0) X(16, 4, 8, 8, 0) X(16, 2, 16, 4, 0) X(16, 4, 8, 4, 0) X(16, 1, 16, 8, 0)             \
  X(16, 1, 16, 4, 0) X(16, 1, 16, 2, 0) X(16, 1, 16, 1, 0) X(16, 1, 4, 1, 0) X(16, 1, 1, 1, 0)             \
  X(8, 2, 16, 8, 0) X(16, 2, 8, 4, 0) X(8, 4, 16, 8, 0)                                                    \
  X(8, 4, 8, 8, 1) X(16, 2, 16, 8, 2) X(8, 4, 16, 8, 2) X(16, 2, 16, 4, 2) X(16, 2, 8, 4, 2) X(16, 2, 16, 4, 4) \
  X(8, 4, 8, 8, 2) X(16, 4, 8, 4, 3)

template <int NS, int R, int NW, int CB, int SEGS>
int launch_int_shape(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                     hipStream_t st, int64_t out_limit, int out_mode) {
  const TileCfg &t = p.fwd;
  const TableLayout L = table_layout(p);
  IntArgs a;
  a.x = (const uint8_t *)d_in;
  a.offs = (const uint32_t *)((const uint8_t *)tables + L.int_offs);
  a.sbase = (const int32_t *)((const uint8_t *)tables + L.int_sbase);
  a.out = d_out;
  a.pitch = p.in_pitch_bytes;
  a.n_samp = p.desc.n_samp;
  a.n_out = out_limit > 0 && out_limit < p.n_out ? out_limit : p.n_out;
  a.out_pitch = out_pitch;
  a.n_chan = p.desc.n_chan;
  a.n_dm = p.desc.n_dm;
  a.row_bytes = t.row_bytes;
  const int64_t tiles_t = (a.n_out + 64 * NS - 1) / (64 * NS);
  const int64_t n_dblk = (p.desc.n_dm + NW * R - 1) / (NW * R);
  if (tiles_t * n_dblk >= ((int64_t)1 << 31)) return (int)hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)(tiles_t * n_dblk)), block(NW * 64);
  const int bits = p.desc.dtype == DD_U4 ? 4 : p.desc.dtype == DD_U16 ? 16 : 8;
  if constexpr (SEGS > 0) {  // phase loads, copy rows within SEGS KiB
    if (t.row_bytes > 1024 * SEGS || (bits == 4 && NS % 8)) return (int)hipErrorInvalidValue;
    const void *fn = bits == 4 ? (const void *)fwd_int_kernel<NS, R, NW, CB, SEGS, 4>
                     : bits == 16
                         ? (out_mode == kOutRawTotals ? (const void *)fwd_int_kernel<NS, R, NW, CB, SEGS, 16, kOutRawTotals>
                            : out_mode == kOutCombineHigh
                                ? (const void *)fwd_int_kernel<NS, R, NW, CB, SEGS, 16, kOutCombineHigh>
                                : (const void *)fwd_int_kernel<NS, R, NW, CB, SEGS, 16>)
                         : (const void *)fwd_int_kernel<NS, R, NW, CB, SEGS, 8>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, t.lds_bytes);
    if (e != hipSuccess) return (int)e;
    if (bits == 4)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, SEGS, 4>), grid, block, t.lds_bytes, st, a, (int)n_dblk,
                         (int)tiles_t, t.order);
    else if (bits == 16 && out_mode == kOutRawTotals)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, SEGS, 16, kOutRawTotals>), grid, block, t.lds_bytes, st, a,
                         (int)n_dblk, (int)tiles_t, t.order);
    else if (bits == 16 && out_mode == kOutCombineHigh)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, SEGS, 16, kOutCombineHigh>), grid, block, t.lds_bytes, st, a,
                         (int)n_dblk, (int)tiles_t, t.order);
    else if (bits == 16)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, SEGS, 16>), grid, block, t.lds_bytes, st, a, (int)n_dblk,
                         (int)tiles_t, t.order);
    else
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, SEGS, 8>), grid, block, t.lds_bytes, st, a, (int)n_dblk,
                         (int)tiles_t, t.order);
    return (int)hipGetLastError();
  } else {
    const void *fn = bits == 4 ? (const void *)fwd_int_kernel<NS, R, NW, CB, 0, 4>
                     : bits == 16
                         ? (out_mode == kOutRawTotals     ? (const void *)fwd_int_kernel<NS, R, NW, CB, 0, 16, kOutRawTotals>
                            : out_mode == kOutCombineHigh ? (const void *)fwd_int_kernel<NS, R, NW, CB, 0, 16, kOutCombineHigh>
                                                          : (const void *)fwd_int_kernel<NS, R, NW, CB, 0, 16>)
                         : (const void *)fwd_int_kernel<NS, R, NW, CB, 0, 8>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, t.lds_bytes);
    if (e != hipSuccess) return (int)e;
    if (bits == 4)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, 0, 4>), grid, block, t.lds_bytes, st, a, (int)n_dblk,
                         (int)tiles_t, t.order);
    else if (bits == 16 && out_mode == kOutRawTotals)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, 0, 16, kOutRawTotals>), grid, block, t.lds_bytes, st, a,
                         (int)n_dblk, (int)tiles_t, t.order);
    else if (bits == 16 && out_mode == kOutCombineHigh)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, 0, 16, kOutCombineHigh>), grid, block, t.lds_bytes, st, a,
                         (int)n_dblk, (int)tiles_t, t.order);
    else if (bits == 16)
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, 0, 16>), grid, block, t.lds_bytes, st, a, (int)n_dblk,
                         (int)tiles_t, t.order);
    else
      hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, CB, 0, 8>), grid, block, t.lds_bytes, st, a, (int)n_dblk,
                         (int)tiles_t, t.order);
    return (int)hipGetLastError();
  }
}

}  // namespace

#define DD_ROW(NS, R, NW, CB, SEGS) {NS, R, NW, CB, SEGS},
const int kIntShapes[][5] = {DD_INT_SHAPES(DD_ROW)};
#undef DD_ROW
const int kNumIntShapes = (int)(sizeof(kIntShapes) / sizeof(kIntShapes[0]));

int launch_forward_int(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                       void *stream, int64_t out_limit, int out_mode) {
  const TileCfg &t = p.fwd;
  if (out_mode != kOutFloat && p.desc.dtype != DD_U16) return (int)hipErrorInvalidValue;
  if (is_direct(t)) return launch_forward_direct(p, tables, d_in, d_out, out_pitch, stream, out_limit, out_mode);
#define DD_TRY(NS, R, NW, CB, SEGS)                                                                    \
  if (t.ns == NS && t.dm_per_wave == R && t.waves == NW && t.chan_block == CB && t.segs == SEGS)       \
    return launch_int_shape<NS, R, NW, CB, SEGS>(p, tables, d_in, d_out, out_pitch, (hipStream_t)stream, out_limit, \
                                                 out_mode);
  DD_INT_SHAPES(DD_TRY)
#undef DD_TRY
  return (int)hipErrorInvalidValue;
}

int batch_kernels(int ns, int dm_per_wave, int waves, int chan_block, int segs, int dtype, int lds_bytes,
                  BatchLaunch *out) {
  const void *fn = nullptr;
#define DD_TRY(NS, R, NW, CB, SEGS)                                                                        \
  if (ns == NS && dm_per_wave == R && waves == NW && chan_block == CB && segs == SEGS)                     \
    fn = SEGS > 0 ? (dtype == DD_U8   ? (const void *)fwd_int_batched_kernel<NS, R, NW, CB, SEGS, 8>         \
                     : dtype == DD_U4 ? (const void *)fwd_int_batched_kernel<NS, R, NW, CB, SEGS, 4>         \
                                      : (const void *)fwd_int_batched_kernel<NS, R, NW, CB, SEGS, 16>)       \
         : dtype == DD_U4  ? (const void *)fwd_int_batched_kernel<NS, R, NW, CB, 0, 4>                     \
         : dtype == DD_U16 ? (const void *)fwd_int_batched_kernel<NS, R, NW, CB, 0, 16>                    \
                           : (const void *)fwd_int_batched_kernel<NS, R, NW, CB, 0, 8>;
  DD_INT_SHAPES(DD_TRY)
#undef DD_TRY
  if (!fn) return (int)hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return (int)e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, waves * 64, lds_bytes);
  if (e != hipSuccess) return (int)e;
  int dev = 0, n_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  out->reset_fn = (const void *)reset_counter_kernel;
  out->main_fn = fn;
  out->grid = n_cu * (per_cu > 0 ? per_cu : 1);
  out->block = waves * 64;
  out->lds_bytes = lds_bytes;
  return 0;
}

}  // namespace dd
