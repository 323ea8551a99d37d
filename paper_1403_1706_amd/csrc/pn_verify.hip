// Validation (Section 3.3): banded bit-parallel semiglobal edit distance,
// one candidate per lane, the band of W = 2k+1 diagonals [d-k, d+k] held in
// one 32-bit word (k <= 15); reads with 15 < k <= 31 take a third pass with
// the band in one 64-bit word (k_verify_wide).
//
// The band is processed row by row (one read letter per step).  Bit b of
// row i stands for column c = i + (d-k) + b, so the same bit index is the
// same diagonal in every row.  The words VP/VN hold the horizontal
// differences D[i][c] - D[i][c-1] (+1 / -1) along the row; a step is Myers'
// bit-vector column update (Myers 1999, in the formulation of Hyyro 2003)
// with the roles of text and pattern exchanged: the band's reference
// letters are the "pattern" bits, the read letter x_i is the "text"
// character.  Between rows the previous row's differences move one bit
// down (its column c sits at bit b+1 of the previous row); the column that
// enters on the right has no value in the band and is given the difference
// +1, and the carry into bit 0 is +1 as well — both stand for paths that
// are never better than the in-band diagonal move, so the band values are
// exactly those of the band-restricted recurrence.
//
// Reference positions outside [0, L) never match (validity plane V): with
// a free start on row 0 this reproduces E[i][0] = i at column 0.  The
// value of the right-most band cell is tracked explicitly; every other
// cell follows from the differences.  A lane stops as soon as every cell of
// its row exceeds k (the row minimum never decreases from one row to the
// next; bounded below by R - #(+1 steps)), or after row n, where it reports
// each end column with value <= k.
//
// Lanes of a wave run in lockstep, so a wave costs as many rows as its
// longest candidate.  Most candidates end within a few rows while true hits
// run the full read, so verification takes two passes: every candidate for
// at most 16 rows, then only the survivors, packed densely, to the end.
// Records and survivors are staged per wave in LDS and appended with one
// atomic per flush to one of kShards output regions.
#include <algorithm>

#include "pn_band.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kStage = 256;  // staged entries per wave
constexpr int kShortRows = 16;    // row cap of the first pass
// waves per SIMD the first pass is compiled for (its registers allow 6 without
// spilling; the second pass keeps the compiler's choice)
constexpr int kFirstWaves = 6;

// Entries (8 bytes) staged per wave in LDS and appended to one output region
// with one global atomic per flush.  A lane that finds the stage full takes
// a global slot of its own.
struct Stage {
    unsigned long long *buf;    // this wave's LDS stage
    uint32_t *cnt;              // this wave's LDS counter
    unsigned long long *region; // output region
    unsigned long long *count;  // its counter
    uint64_t cap;               // its capacity

    __device__ __forceinline__ void push(unsigned long long v) {
        const uint32_t i = atomicAdd(cnt, 1u);
        if (i < kStage) {
            buf[i] = v;
            return;
        }
        const unsigned long long at = atomicAdd(count, 1ull);
        if (at < cap) region[at] = v;
    }

    // whole wave, converged
    __device__ __forceinline__ void flush(int lane) {
        __builtin_amdgcn_wave_barrier();
        const uint32_t n = min(*cnt, kStage);
        if (n == 0) return;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count, (unsigned long long)n);
        base = __shfl(base, 0);
        for (uint32_t i = lane; i < n; i += 64)
            if (base + i < cap) region[base + i] = buf[i];
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) *cnt = 0;
        __builtin_amdgcn_wave_barrier();
    }
};

// A candidate ready to run: its parameters and first memory words.
struct Cand {
    uint2 c;
    bool ok;
    bool wide;  // k > PN_BAND_K: left to the 64-bit band pass
    bool tail;  // first pass: check the read's last rows (reverse complement band)
    int len, k;
    int64_t lo;  // reference position of the band's first diagonal
    const uint4 *pl;
    const uint2 *rp;
    unsigned long long head;  // record key prefix (read, strand)
    PnBandHead hd;
};

// issue a candidate's loads (slot value c; padding and bad reads give !ok).
// With `tail` (first pass, PN_CAND_TAIL) the band is set up for the read's
// reverse complement against the other strand: read letter i on diagonal
// d is reverse-complement letter len-1-i on diagonal L-len-d, so the first
// rows of that band are the last rows of the read's own.
__device__ __forceinline__ void start(const PnRefDev &ref, const PnIndexDev &ix, int kglob,
                                      const uint8_t *__restrict__ kpr, int ebits, uint2 c,
                                      bool first, Cand &x) {
    x.c = c;
    x.ok = false;
    x.wide = false;
    if (c.x == PN_CAND_NONE) return;  // padding slot
    const uint32_t r = c.x & PN_CAND_READ;
    const uint32_t s = c.x >> 31;
    x.tail = first && (c.x & PN_CAND_TAIL);
    x.len = pn_cand_len(c.x);
    x.k = kglob >= 0 ? kglob : (int)kpr[r];
    if (x.k > PN_MAX_K || x.len < 1 || x.len > PN_MAX_READ_LEN) return;
    if (x.k > PN_BAND_K) {
        x.wide = true;
        return;
    }
    x.ok = true;
    const int64_t d = (int64_t)c.y - (int64_t)PN_DBIAS;
    if (x.tail) {
        x.lo = (int64_t)ref.L - x.len - d - x.k;
        x.pl = s ? ref.planes[0] : ref.planes[1];
        x.rp = ix.rplanes_rc + (uint64_t)r * PN_READ_WORDS;
    } else {
        x.lo = d - x.k;
        x.pl = s ? ref.planes[1] : ref.planes[0];
        x.rp = ix.rplanes + (uint64_t)r * PN_READ_WORDS;
    }
    x.head = (((unsigned long long)r << 1) | s) << ebits;
    pn_band_load(x.pl, x.rp, x.lo, x.hd);
}

// Block b reads input region b % in.regions; its records go to output
// region b % kShards and (capped passes) its survivors to long region
// b % in.regions, which can hold every candidate of that input region.
// kFirst: the first pass (16 rows, tail checks); kCapped: the pass stops
// each candidate after `cap` rows and hands the survivors on.
template <bool kFirst, bool kCapped>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kFirst ? kFirstWaves : 1))) void k_verify(PnRefDev ref, PnIndexDev ix, pn::VerifyIn in,
                                                     int kglob, const uint8_t *__restrict__ kpr,
                                                     pn::VerifyOut out, uint2 *longc,
                                                     unsigned long long *n_long, int cap) {
    __shared__ unsigned long long s_rec[kWaves][kStage];
    __shared__ unsigned long long s_long[kCapped ? kWaves : 1][kCapped ? kStage : 1];
    __shared__ uint32_t s_cnt[kWaves][2];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    if (lane == 0) s_cnt[wv][0] = s_cnt[wv][1] = 0;
    __builtin_amdgcn_wave_barrier();
    const uint32_t rin = blockIdx.x % in.regions;
    const uint32_t rout = blockIdx.x % pn::kShards;
    Stage rec{s_rec[wv], &s_cnt[wv][0], out.records + (uint64_t)rout * out.sh.region_cap,
              out.sh.counts + rout, out.sh.region_cap};
    Stage lng{s_long[kCapped ? wv : 0], &s_cnt[wv][1],
              (unsigned long long *)longc + (uint64_t)rin * in.region_cap, n_long + rin,
              in.region_cap};

    const uint2 *cands = in.cands + (uint64_t)rin * in.region_cap;
    const uint64_t n = min((uint64_t)in.counts[rin], in.region_cap);
    const uint64_t per = gridDim.x / in.regions;  // blocks per input region
    const uint64_t stride = per * kThreads;
    const uint2 none = make_uint2(PN_CAND_NONE, PN_CAND_NONE);
    unsigned long long rows = 0;
    // Software pipeline over this lane's candidates: while one candidate's
    // rows run, the next one's read length, k and first plane words are in
    // flight, and the one after that is being read from the list.
    uint64_t base = (blockIdx.x / in.regions) * kThreads + (uint64_t)wv * 64;
    uint2 c_next = base + lane < n ? cands[base + lane] : none;
    uint2 c_after = base + stride + lane < n ? cands[base + stride + lane] : none;
    Cand cur;
    start(ref, ix, kglob, kpr, out.ebits, c_next, kFirst, cur);
    // the loop bound is wave-uniform, so the wave is converged at the flushes
    for (; base < n; base += stride) {
        Cand nxt;
        start(ref, ix, kglob, kpr, out.ebits, c_after, kFirst, nxt);
        const uint64_t ci2 = base + 2 * stride + lane;
        c_after = ci2 < n ? cands[ci2] : none;
        // capped passes: a wave whose reads are all longer than the row cap
        // never reaches a last row (wave-uniform); later passes: no row
        // below the wave's shortest read is a last row
        const int row_cap = kFirst ? kShortRows : kCapped ? cap : PN_MAX_READ_LEN;
        const bool capped = kCapped && __all(!cur.ok || cur.len > row_cap);
        int no_end = 0;
        if (!kFirst) {
            no_end = cur.ok ? cur.len : PN_MAX_READ_LEN + 1;
            for (int o = 32; o > 0; o >>= 1) no_end = min(no_end, __shfl_xor(no_end, o));
            no_end = __builtin_amdgcn_readfirstlane(no_end);
        }
        if (cur.ok) {
            const unsigned long long head = cur.head;
            const bool tail = kFirst && cur.tail;
            auto emit = [&](uint32_t e, int v) {
                if (!tail) rec.push(((head | (unsigned long long)e) << 5) | (unsigned long long)v);
            };
            const int rw =
                capped ? pn_band_run<false>(cur.hd, cur.pl, cur.rp, cur.len, cur.k, cur.lo, ref.L,
                                            row_cap, emit)
                       : pn_band_run(cur.hd, cur.pl, cur.rp, cur.len, cur.k, cur.lo, ref.L,
                                     row_cap, emit, no_end);
            // survivors (and tail checks that reached the read's first
            // letter) run again, forward, from row 0
            if (kCapped && (rw < 0 || (kFirst && tail && rw == cur.len)))
                lng.push(((unsigned long long)cur.c.y << 32) | cur.c.x);
            rows += (unsigned long long)(rw < 0 ? -rw : rw);
        } else if (kCapped && cur.wide) {
            lng.push(((unsigned long long)cur.c.y << 32) | cur.c.x);
        }
        cur = nxt;
        if (*rec.cnt >= kStage / 2) rec.flush(lane);
        if (kCapped && *lng.cnt >= kStage / 2) lng.flush(lane);
    }
    rec.flush(lane);
    if (kCapped) lng.flush(lane);
    for (int o = 32; o > 0; o >>= 1) rows += __shfl_xor(rows, o);
    if (lane == 0 && rows) atomicAdd(out.rows, rows);
}

// The band pass for reads with PN_BAND_K < k <= PN_MAX_K, over the survivor
// list of the first pass (or of the count filter), which holds every such
// candidate: the band of up to 63 diagonals in one 64-bit word, row 0 to
// the end, one candidate per lane.  Such reads are rare (long reads with a
// small q), so the pass has no pipelining of its own.
__global__ __launch_bounds__(kThreads) void k_verify_wide(PnRefDev ref, PnIndexDev ix,
                                                          pn::VerifyIn in, int kglob,
                                                          const uint8_t *__restrict__ kpr,
                                                          pn::VerifyOut out) {
    __shared__ unsigned long long s_rec[kWaves][kStage];
    __shared__ uint32_t s_cnt[kWaves];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    if (lane == 0) s_cnt[wv] = 0;
    __builtin_amdgcn_wave_barrier();
    const uint32_t rin = blockIdx.x % in.regions;
    const uint32_t rout = blockIdx.x % pn::kShards;
    Stage rec{s_rec[wv], &s_cnt[wv], out.records + (uint64_t)rout * out.sh.region_cap,
              out.sh.counts + rout, out.sh.region_cap};
    const uint2 *cands = in.cands + (uint64_t)rin * in.region_cap;
    const uint64_t n = min((uint64_t)in.counts[rin], in.region_cap);
    const uint64_t stride = (uint64_t)(gridDim.x / in.regions) * kThreads;
    unsigned long long rows = 0;
    // the loop bound is wave-uniform, so the wave is converged at the flushes
    for (uint64_t base = (blockIdx.x / in.regions) * kThreads + (uint64_t)wv * 64; base < n;
         base += stride) {
        const uint64_t ci = base + lane;
        const uint2 c = ci < n ? cands[ci] : make_uint2(PN_CAND_NONE, PN_CAND_NONE);
        if (c.x != PN_CAND_NONE) {
            const uint32_t r = c.x & PN_CAND_READ;
            const uint32_t s = c.x >> 31;
            const int len = pn_cand_len(c.x);
            const int k = kglob >= 0 ? kglob : (int)kpr[r];
            if (k > PN_BAND_K && k <= PN_MAX_K && len >= 1 && len <= PN_MAX_READ_LEN) {
                const int64_t d = (int64_t)c.y - (int64_t)PN_DBIAS;
                const unsigned long long head = (((unsigned long long)r << 1) | s) << out.ebits;
                auto emit = [&](uint32_t e, int v) {
                    rec.push(((head | (unsigned long long)e) << 5) | (unsigned long long)v);
                };
                rows += (unsigned long long)pn_band_verify_wide(
                    s ? ref.planes[1] : ref.planes[0], ix.rplanes + (uint64_t)r * PN_READ_WORDS,
                    len, k, d - k, ref.L, emit);
            }
        }
        if (*rec.cnt >= kStage / 2) rec.flush(lane);
    }
    rec.flush(lane);
    for (int o = 32; o > 0; o >>= 1) rows += __shfl_xor(rows, o);
    if (lane == 0 && rows) atomicAdd(out.rows, rows);
}

// The count filter over a candidate list: candidates that may hold a hit
// go to the survivor list (longc, one region per input region), which the
// band pass then runs from row 0 to the end.
// A count-filter candidate ready to run: the H and L words of its first
// four plane blocks and the read's first word (the validity words are
// loaded only for a wave whose bands leave the reference), fewer registers
// than a verification candidate so that more waves fit.
struct CountCand {
    uint2 c;
    int len, k;  // k < 0: nothing to do
    int w0;      // the first read word counted (see count_start)
    int64_t lo;
    uint2 A, B, C, Dn;
    uint2 rw0;
};

__device__ __forceinline__ const uint4 *count_planes(const PnRefDev &ref, uint2 c) {
    return (c.x >> 31) ? ref.planes[1] : ref.planes[0];
}

__device__ __forceinline__ void count_start(const PnRefDev &ref, const PnIndexDev &ix, int kglob,
                                            const uint8_t *__restrict__ kpr, uint2 c,
                                            CountCand &x) {
    x.c = c;
    x.k = -1;
    if (c.x == PN_CAND_NONE) return;
    const uint32_t r = c.x & PN_CAND_READ;
    const int len = pn_cand_len(c.x);
    const int k = kglob >= 0 ? kglob : (int)kpr[r];
    if (k > PN_MAX_K || len < 1 || len > PN_MAX_READ_LEN) return;
    x.len = len;
    x.k = k;
    x.lo = (int64_t)c.y - (int64_t)PN_DBIAS - k;
    // A candidate whose exact window lies in the read's first half
    // (PN_CAND_TAIL) is counted from its last whole read word backwards:
    // the words far from the window decide sooner, and a word that holds
    // the window always shows its pieces.  The pieces past the last whole
    // word are then never counted but taken as found (a keep, never a drop,
    // rests on them), so the count stays lossless.
    const int wf = (len / kPnPiece) / 8;  // whole read words (8 pieces each)
    x.w0 = (c.x & PN_CAND_TAIL) && wf >= 2 ? wf - 1 : 0;
    const uint2 *hl = (const uint2 *)count_planes(ref, c);
    const uint64_t blk = ((uint64_t)(x.lo + PN_PAD_POS) >> 5) + (uint64_t)x.w0;
    x.A = hl[2 * blk];
    x.B = hl[2 * (blk + 1)];
    x.C = hl[2 * (blk + 2)];
    x.Dn = hl[2 * (blk + 3)];
    x.rw0 = ix.rplanes[(uint64_t)r * PN_READ_WORDS + x.w0];
}

// The count filter, one read word per lane and step: a lane whose candidate
// is decided takes its next one at the following step instead of waiting
// for the wave's slowest candidate.  Each lane keeps a candidate in
// progress, the next one with its first memory words already loaded, and
// the candidate word after that (two steps of prefetch, so that its loads
// have a step to land).  A wave takes an even share of its region's
// candidates and hands them out from a wave-wide cursor.
__global__ __launch_bounds__(kThreads) void k_count(PnRefDev ref, PnIndexDev ix, pn::VerifyIn in,
                                                    int kglob, const uint8_t *__restrict__ kpr,
                                                    uint2 *longc, unsigned long long *n_long,
                                                    unsigned long long *letters_out) {
    __shared__ unsigned long long s_long[kWaves][kStage];
    __shared__ uint32_t s_cnt[kWaves];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    if (lane == 0) s_cnt[wv] = 0;
    __builtin_amdgcn_wave_barrier();
    const uint32_t rin = blockIdx.x % in.regions;
    Stage lng{s_long[wv], &s_cnt[wv], (unsigned long long *)longc + (uint64_t)rin * in.region_cap,
              n_long + rin, in.region_cap};
    const uint2 *cands = in.cands + (uint64_t)rin * in.region_cap;
    const uint64_t n = min((uint64_t)in.counts[rin], in.region_cap);
    const uint64_t wpr = (uint64_t)(gridDim.x / in.regions) * kWaves;  // waves of this region
    const uint64_t wr = (uint64_t)(blockIdx.x / in.regions) * kWaves + (uint64_t)wv;
    const uint64_t chunk = (n + wpr - 1) / wpr;
    const uint64_t hi = min(n, wr * chunk + chunk);
    uint64_t cursor = min(n, wr * chunk);  // (wave-uniform) next candidate to hand out
    unsigned long long letters = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    // the candidate word after the next candidate
    bool has_cw = false;
    uint2 cw = make_uint2(PN_CAND_NONE, PN_CAND_NONE);
    // the next candidate, its first words loaded
    bool has_nxt = false;
    CountCand nxt;
    nxt.k = -1;
    // the candidate in progress
    bool has_cur = false;
    uint2 c = make_uint2(0u, 0u);
    uint2 A = c, B = c, C = c, Dn = c, rw = c;
    uint64_t blk = 0;
    uint32_t ph = 0;
    int W = 1, need = 0, found = 0, left = 0, w = 0;
    bool rev = false;  // counting backwards (from word w0 down to 0)
    for (;;) {
        // 1. a lane without a candidate in progress takes the next one
        if (!has_cur && has_nxt) {
            has_nxt = false;
            if (nxt.k >= 0) {
                const int m = nxt.len / kPnPiece;
                const bool inside =
                    nxt.lo >= 0 && nxt.lo + nxt.len + 2 * nxt.k < (int64_t)ref.L;
                if (m - nxt.k <= 0 || !inside || nxt.k > PN_BAND_K) {
                    // nothing to count (too short to drop any, a band that
                    // crosses a reference end, or one wider than the 32
                    // diagonals a text word covers): the band pass settles it
                    lng.push(((unsigned long long)nxt.c.y << 32) | nxt.c.x);
                } else {
                    has_cur = true;
                    c = nxt.c;
                    A = nxt.A;
                    B = nxt.B;
                    C = nxt.C;
                    Dn = nxt.Dn;
                    rw = nxt.rw0;
                    const uint64_t tp = (uint64_t)(nxt.lo + PN_PAD_POS);
                    blk = tp >> 5;
                    ph = (uint32_t)(tp & 31);
                    W = 2 * nxt.k + 1;
                    need = m - nxt.k;
                    left = m;
                    found = 0;
                    w = nxt.w0;
                    rev = nxt.w0 > 0;
                }
            }
        }
        // 2. a lane without a next candidate starts one from its candidate
        //    word, and lanes without a candidate word take new ones
        if (!has_nxt && has_cw) {
            count_start(ref, ix, kglob, kpr, cw, nxt);
            has_nxt = true;
            has_cw = false;
        }
        const bool want = !has_cw && cursor < hi;
        const unsigned long long wm = __ballot(want);
        if (want) {
            const uint64_t idx = cursor + (uint64_t)__popcll(wm & below);
            if (idx < hi) {
                cw = cands[idx];
                has_cw = true;
            }
        }
        cursor = min(hi, cursor + (uint64_t)__popcll(wm));
        if (!__any(has_cur || has_nxt || has_cw)) break;
        // 3. one read word of the candidate in progress
        if (has_cur) {
            // (with one k for every read the diagonal loop's bound is
            // wave-uniform: scalar loop control)
            const uint32_t F = kglob >= 0 ? pn_count_word_hl(A, B, C, rw, ph, 2 * kglob + 1)
                                          : pn_count_word_hl(A, B, C, rw, ph, W);
            // (a backward count takes whole words only)
            found += __popc(F & pn_piece_firsts(rev ? 8 : left));
            const int now = rev || left >= 8 ? 8 : left;
            letters += 32;
            if (found >= need || (rev && w == 0 && found + (left - now) >= need)) {
                lng.push(((unsigned long long)c.y << 32) | c.x);
                has_cur = false;
            } else if (found + (left - now) < need) {
                has_cur = false;
            } else {
                // the next word (the one after, or before when counting
                // backwards): its read plane word and one more text block
                const uint2 *hl = (const uint2 *)count_planes(ref, c);
                const uint2 *rp = ix.rplanes + (uint64_t)(c.x & PN_CAND_READ) * PN_READ_WORDS;
                const int wn = rev ? w - 1 : w + 1;
                rw = rp[wn];
                const uint2 nb = hl[2 * (blk + (uint64_t)(rev ? wn : wn + 3))];
                if (rev) {
                    Dn = C;
                    C = B;
                    B = A;
                    A = nb;
                } else {
                    A = B;
                    B = C;
                    C = Dn;
                    Dn = nb;
                }
                left -= 8;
                w = wn;
            }
        }
        if (*lng.cnt >= kStage / 2) lng.flush(lane);
    }
    lng.flush(lane);
    for (int o = 32; o > 0; o >>= 1) letters += __shfl_xor(letters, o);
    if (lane == 0 && letters) atomicAdd(letters_out, letters);
}

// Candidates in the C ABI's layout (16 bytes: read id u32, strand u8, three
// reserved bytes, diagonal i64) to the verification's (read | strand << 31,
// diagonal + PN_DBIAS) words.  A candidate whose read, strand or diagonal is
// out of range becomes a padding slot and sets bit 3 of *status.
// the length field of a candidate word for read r (false: no verifiable read)
__device__ __forceinline__ bool cand_len_bits(const uint64_t *offsets, uint32_t r, uint32_t &bits) {
    const uint64_t len = offsets[r + 1] - offsets[r];
    bits = (uint32_t)((len - 1) & 0xffu) << PN_CAND_LEN_SHIFT;
    return len >= 1 && len <= PN_MAX_READ_LEN;
}

__global__ __launch_bounds__(256) void k_cands_in(const uint4 *__restrict__ in, uint64_t n,
                                                  uint32_t n_reads, uint64_t L,
                                                  const uint64_t *__restrict__ offsets,
                                                  uint2 *__restrict__ out, uint32_t *status) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 v = in[i];
    const uint32_t strand = v.y & 0xffu;
    const int64_t d = (int64_t)(((uint64_t)v.w << 32) | v.z);
    const bool ok = v.x < n_reads && strand <= 1u && d >= -(int64_t)PN_MAX_READ_LEN &&
                    d <= (int64_t)L;
    if (!ok) atomicOr(status, 8u);
    uint32_t lb = 0;
    const bool has_len = ok && cand_len_bits(offsets, v.x, lb);
    out[i] = has_len ? make_uint2(v.x | lb | (strand << 31), (uint32_t)(d + (int64_t)PN_DBIAS))
                     : make_uint2(PN_CAND_NONE, PN_CAND_NONE);
}

__global__ __launch_bounds__(256) void k_cands_len(uint2 *__restrict__ c, uint64_t n,
                                                   const uint64_t *__restrict__ offsets) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint2 v = c[i];
        if (v.x == PN_CAND_NONE) continue;
        uint32_t lb = 0;
        c[i] = cand_len_bits(offsets, v.x & PN_CAND_READ, lb)
                   ? make_uint2(v.x | lb, v.y)
                   : make_uint2(PN_CAND_NONE, PN_CAND_NONE);
    }
}

}  // namespace

namespace pn {

void launch_verify(const PnRefDev &ref, const PnIndexDev &ix, VerifyIn in, int kglob,
                   const uint8_t *kpr, VerifyOut out, uint2 *longc, unsigned long long *n_long,
                   bool first, hipStream_t st) {
    if (!in.region_cap || !in.regions) return;
    // blocks: a multiple of the input regions, enough to fill the chip
    uint64_t per = (in.region_cap + kThreads - 1) / kThreads;
    const uint64_t max_per = std::max<uint64_t>(8192 / in.regions, 1);
    if (per > max_per) per = max_per;
    const dim3 grid((unsigned)(per * in.regions));
    if (first) {
        hipLaunchKernelGGL((k_verify<true, true>), grid, dim3(kThreads), 0, st, ref, ix, in, kglob,
                           kpr, out, longc, n_long, kShortRows);
    } else {
        VerifyIn in2{longc, n_long, in.regions, in.region_cap};
        hipLaunchKernelGGL((k_verify<false, false>), grid, dim3(kThreads), 0, st, ref, ix, in2,
                           kglob, kpr, out, longc, n_long, PN_MAX_READ_LEN);
    }
}

void launch_verify_wide(const PnRefDev &ref, const PnIndexDev &ix, VerifyIn in, int kglob,
                        const uint8_t *kpr, VerifyOut out, hipStream_t st) {
    if (!in.region_cap || !in.regions) return;
    uint64_t per = (in.region_cap + kThreads - 1) / kThreads;
    const uint64_t max_per = std::max<uint64_t>(8192 / in.regions, 1);
    if (per > max_per) per = max_per;
    hipLaunchKernelGGL(k_verify_wide, dim3((unsigned)(per * in.regions)), dim3(kThreads), 0, st,
                       ref, ix, in, kglob, kpr, out);
}

void launch_count(const PnRefDev &ref, const PnIndexDev &ix, VerifyIn in, int kglob,
                  const uint8_t *kpr, uint2 *surv, unsigned long long *n_surv,
                  unsigned long long *letters, hipStream_t st) {
    if (!in.region_cap || !in.regions) return;
    uint64_t per = (in.region_cap + kThreads - 1) / kThreads;
    const uint64_t max_per = std::max<uint64_t>(8192 / in.regions, 1);
    if (per > max_per) per = max_per;
    hipLaunchKernelGGL(k_count, dim3((unsigned)(per * in.regions)), dim3(kThreads), 0, st, ref,
                       ix, in, kglob, kpr, surv, n_surv, letters);
}

void launch_cands_in(const void *in, uint64_t n, uint32_t n_reads, uint64_t L,
                     const uint64_t *offsets, uint2 *out, uint32_t *status, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_cands_in, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const uint4 *)in, n, n_reads, L, offsets, out, status);
}

void launch_cands_len(uint2 *cands, uint64_t n, const uint64_t *offsets, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_cands_len, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, cands, n,
                       offsets);
}

}  // namespace pn
