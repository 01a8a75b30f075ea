// mrpsim: spectral kinetic simulation of the ideal Multipole Resonance Probe
// (Gong, Friedrichs, Oberrath, Brinkmann, arXiv:2111.13072) on one MI355X
// (gfx950).  C ABI declared in include/mrpsim.h.
//
// One time step (Sec. 3 field solver + Sec. 4 pusher) runs as these kernels:
//   sort:    key (r^2, id) -> bucket histogram -> bucket offsets -> scatter
//            -> exact rank inside each bucket -> permuted SoA copy
//   moments: per tile of 64 radially consecutive particles, the sums of
//            q R_lm (regular solid harmonics) and q I_lm (irregular ones)
//   carries: exclusive prefix of the interior sums and exclusive suffix of
//            the exterior sums over tiles, totals T_lm, the boundary (image)
//            response, the surface charge, the hemisphere drive and Q_diff
//   field:   per particle, the far field of all other tiles from the tile's
//            coefficient vector, the near field of its own tile pair by pair,
//            the self-image correction and the ion background; then the
//            leapfrog kick/drift, the wall rules and the next step's sort key
//            and bucket slot (the key kernel keys only what the push did not)
// A handle holds one or more independent simulations ("members") that share
// the probe geometry, the truncation l_max and the precision.  Each member
// owns a tile-aligned range of particle slots, a range of carry chunks and a
// range of sort buckets; every kernel maps its tile, chunk or bucket to the
// member through a device table, so one launch of each kernel steps all
// members, and members can be admitted and retired between steps.  A
// member's arithmetic does not depend on the others.  All work is on the
// handle's stream; one step is captured once into a HIP graph and replayed.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <utility>
#include <vector>

#include "mrpsim.h"

namespace {

constexpr double kQ = -1.0;   // electron charge, units of e (Sec. 4)
constexpr double kM = 1.0;    // electron mass, units of m_e
// A particle whose id has this bit set is an ion: charge +1, mass ion_mass.
constexpr uint32_t kIonBit = 0x80000000u;
constexpr double kPi = 3.14159265358979323846;
constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxL = 64;
// A tile (one wave's 64 radially consecutive particles) is two halves of 32:
// the pair sums of the near field run inside a half, and the moments are
// summed per half.  A group is the four tiles of one workgroup of the moments
// and field kernels (256 slots): the carry scan runs over groups, and a
// member's particle slots are whole groups.
constexpr int kHalf = kWave / 2;
constexpr int kTilesPerGroup = kWavesPerBlock;
constexpr int kGroupSlots = kTilesPerGroup * kWave;
// Groups per chunk of the carry scan, per member: a power of two in
// [kChunkMin, kChunkMax], about a member's groups / kChunkTarget, so that small
// members get short serial chains and large ones few chunks.
constexpr int kChunkMin = 8, kChunkMax = 64, kChunkTarget = 256;
constexpr int kScanPerBlock = 1024;  // histogram entries per block of the bucket scan
constexpr int kBucketOccupancy = 8;  // mean particles per sort bucket

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

// ---------------------------------------------------------------------------
// Device-side structures
// ---------------------------------------------------------------------------

// Sorted state (this step's radial order), one array per component: the
// moments and field kernels read it with unit stride.
struct State {
    double *x, *y, *z, *vx, *vy, *vz;
    uint32_t *uid;
};

// Unsorted state (after the push, in the previous step's order): one 64-byte
// record per particle, so the sort's gather of a particle from its scattered
// source slot is a single cache line.
struct alignas(64) PRec {
    double x, y, z, vx, vy, vz;
    uint32_t uid, pad[3];
};

// Per-member control block in device memory.
struct Ctl {
    int64_t step;       // absolute step of the state held in A
    uint32_t n_cur;     // records in A (some may be flagged absorbed)
    uint32_t n_live;    // alive particles sorted into B this step
    uint32_t n_dead;    // particles absorbed so far (graveyard fill)
    uint32_t n_dead_ion;  // of which ions
    double q_surface;   // Q_S used by this step's field
    // the step whose sort keys, bucket slots and bucket counts the last push
    // already produced (-1: none; the key kernel computes them)
    int64_t keys_for = -1;
};

// Per-member description (device table, written by the host between steps).
struct Seg {
    uint32_t p0, cap;   // particle slots [p0, p0 + cap); p0 is a multiple of 256
    uint32_t t0, nt;    // tiles [t0, t0 + nt), t0 = p0 / 64
    uint32_t g0, ng;    // groups [g0, g0 + ng), g0 = p0 / 256
    uint32_t c0, nc;    // carry chunks [c0, c0 + nc)
    uint32_t cl;        // groups per chunk
    uint32_t b0, nb;    // sort buckets [b0, b0 + nb)
    double inv_vol;     // 1 / (r_out^3 - 1)
    double ntilde, inv_ntilde, ion_density, q_surface0, dt, r_out;
    uint64_t seed;
    int32_t probe_bc, wall_bc;
    int64_t n_steps;
    const double *u_asy;
    double *qdiff;
    // optional ion profile: densities at ion_k + 1 equally spaced radii from 1
    // to r_out, then the enclosed ion charge at those radii (super-particle units)
    const double *ion_tab;
    double ion_h, ion_inv_h;
    double ion_qm;      // charge / mass of ion particles (+1 / ion_mass)
    int32_t ion_k;
    int32_t near_w;     // particles of a near-field block: 32 (a half tile) or 64 (the tile)
    int32_t used;
};

constexpr uint32_t kNone = 0xffffffffu;

// Per-l and per-(l, m) constant tables (host-computed, read-only).  The
// super-particle density 1 / ntilde is a per-member factor applied at use.
struct Tables {
    const double *ftil;     // image coefficient f_l, with f_0 = 0 (floating probe)
    const double *wl;       // 1 / (2l+1)
    const double *drive_w;  // c_l b^P_l sqrt(4 pi / (2l+1)) for odd l, else 0
    const double *self_w;   // f_l / (4 pi)
    const double *nfA;      // (2l+1)/(l+1)
    const double *nfB;      // l/(l+1)
    const double4 *nf4;     // {(2l+1)/(l+1), l/(l+1), 2l+1, l}, one wide load per l
    const int *chl;         // degree l of each channel in stream order
    // per channel: the factor that turns a sum of rescaled harmonics (Qh) into
    // a field coefficient, N_lm^2 / (2l+1) (times 1 / ntilde at use)
    const double *chg;
    // Legendre constants of the full near field, per l: {c_l, l c_l,
    // gamma_{l+1}, (2l+1) c_l}, where P_l = c_l Ph_l and the rescaled
    // polynomials obey Ph_{l+1} = u Ph_l - gamma_{l+1} Ph_{l-1}
    const double4 *lg4;
    // Rescaled harmonic recurrence in stream order of (m, l) (m outer,
    // l = m..L inner, so a loop over (m, l) reads consecutive entries): the
    // moments and the far field use Qh_l^m = Q_l^m / N_lm with Qh_m^m = 1,
    // Qh_l^m = z Qh_{l-1}^m - gamma_lm r^2 Qh_{l-2}^m; entries {gamma_lm,
    // l - m, l + m + 1, 0}, one zero entry after the triangle.  The tile sums
    // are sums of Qh; the carries apply N_lm (chn, per channel) twice: once to
    // turn the sums into true moments, once for the field's Qh.
    const double4 *fq4;
    const double *chn;
    // FP32 copies of the field kernel's tables for the FP32-compensated mode
    const float4 *nf4_32;
    const float4 *lg4_32;
    const float4 *fq4_32;
    // FP32 near field's Legendre recurrence on D_l = P_l - P_{l-1}, per l:
    // {l / (l+1), -(2l+1) / (l+1), 2l+1, l+1}
    const float4 *lw4_32;
};

// Channels are kept in "stream order": m = 0..m_top outer, l = max(m,1)..L
// inner, cos then sin for m > 0.  l = 0 has no channel: its field is Gauss's
// law over the radial order (computed in the field kernel).
struct KParams {
    int L;          // l_max
    int C;          // channels: (L+1)^2 - 1 (full) or L (axisymmetric)
    int C2;         // 2C: interior then exterior
    int SW;         // C2 + 1: group sums also carry the group's total charge
    int HW;         // 4C + 2: a tile's row of H (interior and exterior sums
                    // of the group's other tiles, of its own halves, charges)
    int n_tiles;    // tile capacity (particle slots / 64, a multiple of 4)
    int n_groups;   // n_tiles / 4
    int n_chunks;   // chunk capacity
    int nb;         // bucket capacity
    int n_members;  // member table size
    int fp32;       // SIM_FP32_COMP
    int field_only; // evaluation without a step: every used member runs
    int fuse_keys;  // the push prepares the next step's sort records
};

// The push's tail takes over the key pass from this many tiles on: the
// tail's atomic round trip costs ~3 us per step on a small launch (1e4
// particles: 0.0658 -> 0.0674 ms), the key pass it replaces ~30 ns per
// thousand particles plus its launch (2e6: 64 us against 16 in the push).
constexpr int kFuseKeysMinTiles = 2048;

// Device tables shared by the kernels.
struct Map {
    const Seg *seg;
    Ctl *ctl;
    const uint32_t *tile_member;   // [n_tiles], kNone for free tiles
    const uint32_t *chunk_member;  // [n_chunks], kNone for free chunks
};

// Charge of the immobile ions of a radial profile inside radius r, in
// super-particle units: the density is linear in r on each segment
// [r_j, r_j + h], integrated in closed form in the offset dd = r - r_j.
// (A uniform background enters the field kernel as its field directly.)
__device__ inline double ion_enclosed(const Seg &sg, double r, double r2)
{
    constexpr double kFourPi = 4.0 * 3.14159265358979323846;
    (void)r2;
    const int K = sg.ion_k;
    int j = (int)((r - 1.0) * sg.ion_inv_h);
    j = max(0, min(j, K - 1));
    const double rj = 1.0 + (double)j * sg.ion_h;
    const double dd = r - rj;
    const double nj = sg.ion_tab[j];
    const double beta = (sg.ion_tab[j + 1] - nj) * sg.ion_inv_h;
    const double d2 = dd * dd;
    const double seg = nj * (rj * rj * dd + rj * d2 + d2 * dd / 3.0) +
                       beta * (rj * rj * d2 / 2.0 + 2.0 * rj * d2 * dd / 3.0 + d2 * d2 / 4.0);
    return sg.ion_tab[K + 1 + j] + kFourPi * sg.ntilde * seg;
}

// A member takes part in this launch: it is in use and has steps left (or
// the launch only evaluates the field).
__device__ inline bool member_runs(const Seg &sg, const Ctl &c, const KParams &kp)
{
    return sg.used && (kp.field_only || c.step < sg.n_steps);
}

__host__ __device__ inline int tri(int l, int m) { return l * (l + 1) / 2 + m; }

__device__ inline uint32_t uniform_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Blocks are placed on the 8 XCDs round-robin (block b on XCD b % 8), and
// each XCD has its own L2.  Kernels whose neighbouring blocks share cache
// lines renumber their blocks so that every XCD walks one contiguous range.
constexpr uint32_t kXcds = 8;

__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nblocks)
{
    const uint32_t q = nblocks / kXcds, r = nblocks % kXcds;
    const uint32_t x = b % kXcds, k = b / kXcds;
    return x * q + min(x, r) + k;
}

// Read of a table that no kernel writes while it runs, through the constant
// address space: a wave-uniform index then becomes a scalar load through the
// scalar cache even where the kernel stores to global memory in between
// (which keeps the compiler from proving the read invariant).
template <typename T>
__device__ inline T ld_const(const T *p, int i)
{
    return reinterpret_cast<const __attribute__((address_space(4))) T *>(
        reinterpret_cast<uintptr_t>(p))[i];
}


// r^2 as (x*x + y*y) + z*z without contraction: the exact radial sort key.
__device__ inline double key_r2(double x, double y, double z)
{
    return __dadd_rn(__dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y)), __dmul_rn(z, z));
}

// ---------------------------------------------------------------------------
// Sort: exact order by (r^2, id) through volume-uniform buckets
// ---------------------------------------------------------------------------

// Bucket of a key: a monotone non-decreasing map of r^2 to the member's
// buckets [b0, b0 + nb) by enclosed shell volume.  The sort and the rank
// kernels both use this one expression, so they agree bit for bit.
__device__ inline uint32_t bucket_of(double r2, double inv_vol, uint32_t b0, uint32_t nb)
{
    const double t = (r2 * sqrt(r2) - 1.0) * inv_vol * (double)nb;
    uint32_t lb;
    if (!(t > 0.0)) lb = 0;
    else if (!(t < (double)(nb - 1))) lb = nb - 1;
    else lb = (uint32_t)t;
    return b0 + lb;
}

// Sort records: (key, bucket, slot in the bucket) per particle slot, then
// (key, id, source slot) per position in bucket order; one 16-byte access each.
struct alignas(16) KeyRec {
    uint64_t key;
    uint32_t uid, sub;   // sub = kNone: not sorted this step
};
struct alignas(16) OrdRec {
    uint64_t key;
    uint32_t uid, idx;
};

// Key, bucket and slot inside the bucket, over all particle slots.  One
// step moves a particle across ~10^2 buckets, so the lanes of a wave land in
// almost distinct buckets: each takes its slot with its own atomic add.
// Members whose last push already produced this step's records (keys_for)
// are skipped: the push kernel's tail does the same work for the particles
// it moves, where the field's arithmetic hides the atomics' latency.
__global__ void k_sort_key(Map mp, const PRec *A, const uint8_t *dead, KeyRec *krec,
                           uint32_t *hist, KParams kp)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t tile = i >> 6;
    if ((int)tile >= kp.n_tiles) return;   // whole waves: i < 64 * n_tiles
    const uint32_t mb = uniform_u32(mp.tile_member[tile]);
    bool live = false;
    double inv_vol = 0.0;
    uint32_t b0 = 0, nb = 1;
    if (mb != kNone) {
        const Seg &sg = mp.seg[mb];
        const Ctl &c = mp.ctl[mb];
        if (member_runs(sg, c, kp)) {
            if (c.keys_for == c.step) return;   // wave-uniform
            live = (i - sg.p0) < c.n_cur && !dead[i];
            inv_vol = sg.inv_vol;
            b0 = sg.b0;
            nb = sg.nb;
        }
    }
    KeyRec rec{0ull, 0u, kNone};
    if (live) {
        const double r2 = key_r2(A[i].x, A[i].y, A[i].z);
        rec.key = (uint64_t)__double_as_longlong(r2);
        rec.uid = A[i].uid;
        rec.sub = atomicAdd(&hist[bucket_of(r2, inv_vol, b0, nb)], 1u);
    }
    krec[i] = rec;
}

// Exclusive scan of a u32 array of length n into out[0..n], out[n] = total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kWavesPerBlock];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_a(const uint32_t *in, uint32_t *bsum, int n)
{
    const int base = blockIdx.x * kScanPerBlock;
    uint32_t s = 0;
    for (int k = threadIdx.x; k < kScanPerBlock; k += kBlock) {
        int i = base + k;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Offsets of the buckets: each block adds the sums of the blocks before it
// (at most a few thousand, read from L2) to the scan of its own entries.
// The histogram's last reader: it leaves the histogram zeroed for the next
// step (the handle zeroes it once at creation).
__global__ __launch_bounds__(kBlock) void k_scan_c(uint32_t *in, const uint32_t *bsum,
                                                   uint32_t *out, int n)
{
    uint32_t before = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kBlock) before += bsum[k];
    uint32_t carry;
    block_exclusive_scan(before, &carry);
    constexpr int per = kScanPerBlock / kBlock;
    const int base = blockIdx.x * kScanPerBlock + threadIdx.x * per;
    uint32_t v[per];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        s += v[k];
    }
#pragma unroll
    for (int k = 0; k < per; ++k)
        if (base + k < n) in[base + k] = 0u;
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < per; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
        if (base + k == n - 1) out[n] = run;
    }
}

// The same offsets from one block, walking the histogram kScanPerBlock entries
// at a time with a running carry: for histograms of a few blocks' length it
// replaces the two kernels above by one launch (small runs are launch-bound).
constexpr int kScanSingleMaxBlocks = 4;

__global__ __launch_bounds__(kBlock) void k_scan_single(uint32_t *in, uint32_t *out, int n)
{
    constexpr int per = kScanPerBlock / kBlock;
    uint32_t carry = 0;
    for (int base0 = 0; base0 < n; base0 += kScanPerBlock) {
        const int base = base0 + threadIdx.x * per;
        uint32_t v[per];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < per; ++k) {
            v[k] = (base + k < n) ? in[base + k] : 0u;
            s += v[k];
        }
#pragma unroll
        for (int k = 0; k < per; ++k)
            if (base + k < n) in[base + k] = 0u;
        uint32_t tot;
        uint32_t run = carry + block_exclusive_scan(s, &tot);
#pragma unroll
        for (int k = 0; k < per; ++k) {
            if (base + k < n) out[base + k] = run;
            run += v[k];
            if (base + k == n - 1) out[n] = run;
        }
        carry += tot;
    }
}

// Per member: alive count (its buckets' share of the global offsets) and the
// surface charge Q_S = q_surface0 + the charge absorbed so far, which enters
// the field as an interior l = 0 charge (Q_S / (4 pi r), Sec. 3).  Done by
// the first block of the rank kernel (after the offsets, before the moments).
__device__ inline void member_live(const Map &mp, const uint32_t *off, const KParams &kp)
{
    for (int s = threadIdx.x; s < kp.n_members; s += blockDim.x) {
        const Seg &sg = mp.seg[s];
        Ctl &c = mp.ctl[s];
        if (!member_runs(sg, c, kp)) continue;
        c.keys_for = -1;   // this step's sort records are consumed
        c.n_live = off[sg.b0 + sg.nb] - off[sg.b0];
        c.q_surface =
            (sg.q_surface0 + kQ * (double)(c.n_dead - c.n_dead_ion)) + (double)c.n_dead_ion;
    }
}

// Bucket order (arbitrary inside a bucket): key, id and source slot.  Only
// the records of running members' first n_cur slots count (the push writes
// records for the slots it moves, and slots past the alive count may hold
// older ones).
__global__ void k_sort_scatter(Map mp, const KeyRec *krec, const uint32_t *off, OrdRec *orec,
                               KParams kp)
{
    const uint32_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)kp.n_tiles * kWave) return;
    const KeyRec r = krec[i];   // in bounds; issued before the member's tables
    const uint32_t mb = uniform_u32(mp.tile_member[i >> 6]);
    if (mb == kNone) return;
    const Seg &sg = mp.seg[mb];
    const Ctl &c = mp.ctl[mb];
    if (!member_runs(sg, c, kp) || (i - sg.p0) >= c.n_cur) return;
    if (r.sub == kNone) return;
    // the bucket again, from the key and the member of this slot's tile (the
    // same arithmetic as in the key kernel and the push, so the same bucket)
    const uint32_t b = bucket_of(__longlong_as_double((long long)r.key), sg.inv_vol, sg.b0, sg.nb);
    orec[off[b] + r.sub] = OrdRec{r.key, r.uid, i};
}

// Final position = bucket start + number of bucket mates with a smaller
// (r^2, id) key (independent of the order inside the bucket), moved into the
// member's slot range; the particle's state moves there.  A block's positions
// cover a window of whole buckets, staged in LDS when it fits (12 KB; with
// 24 KB, six blocks per CU, the kernel took 5% longer).
constexpr int kRankWindow = 1024;

__device__ inline uint32_t bucket_of_rec(const Map &mp, const OrdRec &r)
{
    const Seg &sg = mp.seg[mp.tile_member[r.idx >> 6]];
    return bucket_of(__longlong_as_double((long long)r.key), sg.inv_vol, sg.b0, sg.nb);
}

__global__ __launch_bounds__(kBlock) void k_sort_rank_move(Map mp, const OrdRec *orec,
                                                           const uint32_t *off, const PRec *A,
                                                           State B,
                                                           KParams kp)
{
    __shared__ uint64_t wkey[kRankWindow];
    __shared__ uint32_t wuid[kRankWindow];
    if (blockIdx.x == 0) member_live(mp, off, kp);
    const uint32_t n = off[kp.nb];   // alive particles of all running members
    const uint32_t p0 = xcd_block(blockIdx.x, gridDim.x) * kBlock;
    if (p0 >= n) return;
    const uint32_t p_last = min(p0 + kBlock, n) - 1;
    const uint32_t p = p0 + threadIdx.x;
    const bool act = p < n;
    // This lane's record, then its member's tables, its bucket's bounds and
    // the gathered state: all issued before the block's window is staged, so
    // that their round trips overlap the window's (lanes past n take the
    // block's last record and leave after the barrier).
    const OrdRec me = orec[act ? p : p_last];
    const Seg &sg = mp.seg[mp.tile_member[me.idx >> 6]];
    const PRec a = A[me.idx];
    const uint32_t b = bucket_of(__longlong_as_double((long long)me.key), sg.inv_vol, sg.b0, sg.nb);
    const uint32_t lo = off[b], hi = off[b + 1];
    const uint32_t d0 = sg.p0 - off[sg.b0];   // the member's first slot, less its first offset
    const uint32_t w0 = off[bucket_of_rec(mp, orec[p0])];
    const uint32_t w1 = off[bucket_of_rec(mp, orec[p_last]) + 1];
    const bool staged = (w1 - w0) <= (uint32_t)kRankWindow;
    if (staged) {
        for (uint32_t j = w0 + threadIdx.x; j < w1; j += kBlock) {
            const OrdRec r = orec[j];
            wkey[j - w0] = r.key;
            wuid[j - w0] = r.uid;
        }
    }
    __syncthreads();
    if (!act) return;
    const uint64_t k = me.key;
    const uint32_t u = me.uid;
    uint32_t rank = 0;
    if (staged) {
        for (uint32_t j = lo - w0; j < hi - w0; ++j) {
            const uint64_t kj = wkey[j];
            rank += (kj < k) || (kj == k && wuid[j] < u);
        }
    } else {
        for (uint32_t j = lo; j < hi; ++j) {
            const OrdRec rj = orec[j];
            rank += (rj.key < k) || (rj.key == k && rj.uid < u);
        }
    }
    const uint32_t d = d0 + (lo + rank);
    B.x[d] = a.x;
    B.y[d] = a.y;
    B.z[d] = a.z;
    B.vx[d] = a.vx;
    B.vy[d] = a.vy;
    B.vz[d] = a.vz;
    B.uid[d] = u;
}

// ---------------------------------------------------------------------------
// Moments: per-tile sums of q R_lm and q I_lm
// ---------------------------------------------------------------------------
//
// Real solid harmonics through the polynomial Q_l^m(z, r^2) = r^l P~_l^m /
// (r sin th)^m and (x + i y)^m = C_m + i S_m:
//   R_lm^c = Q_l^m C_m,  R_lm^s = Q_l^m S_m,  I_lm = r^-(2l+1) R_lm,
// normalised so that sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b).  The
// kernel sums the rescaled Qh_l^m = Q_l^m / N_lm (a three-operation
// recurrence); the carries restore N_lm.

// A slot holds two channels, one LDS row each: the wave's 64 lanes after the
// fold across 16-lane rows, four quarter rows of 16 partial sums: interior of
// half 0 (lanes 0-15), exterior of half 0 (16-31), interior of half 1 (32-47)
// and exterior of half 1 (48-63), quarter q at row offset q * kQuarterOff.  A
// batch of kSlots slots is read back by pairs of lanes, each pair summing one
// quarter row (kPartials entries each, then one lane exchange).  With
// kQuarterOff = 17 and kRowLen = 68 the 16 lanes of each quarter of the wave
// start their reads on distinct banks.
constexpr int kSlots = 4;                          // slots per batch
constexpr int kQuarterOff = 17;
constexpr int kRowLen = 4 * kQuarterOff;
constexpr int kPartials = 8;                       // entries per lane: 16 / 2
static_assert(kWave == 2 * (2 * kSlots) * 4, "one lane pair per quarter row of a batch");

// Orders this wave's LDS accesses at this point: LDS instructions of one wave
// complete in issue order, so rows a wave wrote are visible to its later
// reads without a block barrier; the fences keep the compiler from moving
// LDS accesses across.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exchange the odd 16-lane rows of a with the even rows of b: afterwards a
// holds the rows {a0, b0, a2, b2} and b the rows {a1, b1, a3, b3}.
__device__ inline void swap_rows16(double &a, double &b)
{
    const uint64_t ua = (uint64_t)__double_as_longlong(a), ub = (uint64_t)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi =
        __builtin_amdgcn_permlane16_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
    a = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | (uint64_t)lo[0]));
    b = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | (uint64_t)lo[1]));
}

// The value of another lane of this lane's quad, through DPP: kPerm is a
// quad_perm control (0xB1: lane xor 1, 0x4E: lane xor 2).  A quad
// permutation has a source for every lane, so no "old" value is needed.
template <int kPerm>
__device__ inline double dpp_quad(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t plo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, kPerm, 0xF, 0xF, true);
    const uint32_t phi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), kPerm, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)phi << 32) | plo));
}

// A tile's row of H: [interior | interior, half 0 | exterior | exterior,
// half 1 | charge, unused]: the interior sums of the group's tiles before
// this one, the halves' own sums (a half's coefficients take the other half's
// part from them), the exterior sums of the group's tiles after this one, and
// the charge of the group's tiles before this one.

// The value of lane + 4 within its row of 16 lanes (DPP row_shl:4; the last
// four lanes of a row read zero).
__device__ inline double dpp_row_shl4(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t plo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x104, 0xF, 0xF, true);
    const uint32_t phi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x104, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)phi << 32) | plo));
}

template <bool FULL>
__global__ __launch_bounds__(kBlock, 8) void k_moments(Map mp, State B, Tables tb, KParams kp,
                                                    double *H, double *GS)
{
    // Per wave (one tile of 64 particles), the sums of q R (interior) and
    // q I (exterior) of every channel over each half of the tile, in a tree:
    //  1. R and I of one channel are folded across 16-lane rows (lanes 0-15
    //     then hold R over particle pairs of half 0, lanes 16-31 I of half 0,
    //     lanes 32-63 the same for half 1), and the result is one LDS row of a
    //     slot; a slot holds two channels (cos and sin of one (l, m), or two
    //     degrees of m = 0);
    //  2. every kSlots slots each pair of lanes sums one quarter row
    //     (kPartials entries each, then a lane exchange); the pairs of half 0
    //     add half 1's sum from four lanes on (the whole-tile sums), and the
    //     halves' own sums (interior of half 0, exterior of half 1) go to the
    //     tile's row of H;
    //  3. every kXBatches batches the four waves of the block (the group's
    //     tiles) trade their whole-tile sums through LDS, one channel and
    //     side per lane: each stores in its tile's row of H the interior
    //     sums of the tiles before it and the exterior sums of those after
    //     it; the last and first wave store the group's interior and
    //     exterior totals in its row of the carry scan (GS: interior,
    //     exterior, charge).
    // The m = 0 block is padded to an even count with a zero channel, so a
    // slot always holds two positions of the padded channel order.
    __shared__ double buf[kWavesPerBlock][kSlots * 2 * kRowLen];
    // whole-tile sums of kXBatches batches, per wave (interior, exterior):
    // one channel and side per lane of an exchange (one set, with a barrier
    // before and after its reads, keeps eight waves per SIMD)
    constexpr int kXBatches = 4;
    constexpr int kXLen = kXBatches * 2 * kSlots;
    static_assert(2 * kXLen <= kWave, "one channel and side per lane in an exchange");
    __shared__ double xch[kWavesPerBlock][2][kXLen];
    __shared__ double qx[kWavesPerBlock];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const uint32_t group = blockIdx.x;
    const uint32_t tile = uniform_u32(group * kTilesPerGroup + w);
    // the member (the same for the group's four tiles: a member's slots are
    // whole groups); n = its alive count, lt = the tile's index in it
    bool tile_ok = false, halves = false;
    uint32_t n = 0, lt = 0;
    if ((int)tile < kp.n_tiles) {
        const uint32_t mb = uniform_u32(mp.tile_member[tile]);
        if (mb != kNone && member_runs(mp.seg[mb], mp.ctl[mb], kp)) {
            tile_ok = true;
            n = mp.ctl[mb].n_live;
            lt = tile - mp.seg[mb].t0;
            // the halves' own sums only where the field kernel uses them
            halves = uniform_u32((uint32_t)mp.seg[mb].near_w) == (uint32_t)kHalf;
        }
    }
    const uint32_t p = tile * kWave + lane;
    const bool valid = tile_ok && lt * kWave + lane < n;
    double x = 0.0, y = 0.0, z = 2.0;
    bool ion = false;
    if (valid) {
        x = B.x[p];
        y = B.y[p];
        z = B.z[p];
        ion = (B.uid[p] & kIonBit) != 0;
    }
    const double q = valid ? (ion ? 1.0 : kQ) : 0.0;
    const double r2 = x * x + y * y + z * z;
    const double inv_r2 = 1.0 / r2;
    const double inv_r = 1.0 / sqrt(r2);
    const int L = kp.L;
    const int C = kp.C;
    double *Ht = H + (size_t)tile * kp.HW;
    double *Gs = GS + (size_t)group * kp.SW;
    {
        // the tile's charge (exact: counts of ions and electrons), then the
        // group's tiles before this one (in tile order) and the group's total
        const uint64_t vb = __ballot(valid), ib = __ballot(valid && ion);
        const int n_val = __popcll(vb), n_ion = __popcll(ib);
        if (lane == 0) qx[w] = (double)n_ion + kQ * (double)(n_val - n_ion);
        __syncthreads();
        if (tile_ok && lane == 0) {
            double sq = 0.0;
            for (int k = 0; k < w; ++k) sq += qx[k];
            Ht[4 * C] = sq;
            if (w == kWavesPerBlock - 1) Gs[kp.C2] = sq + qx[w];
        }
    }

    double *wb = buf[w];
    // writer: lane -> its entry of a row
    double *wr = wb + (lane >> 4) * kQuarterOff + (lane & 15);
    // reader: lane pair v = 4 rr + rq (row rr = 2 s + j of the batch: slot s,
    // its channel j; quarter rq) sums that quarter row; part t of it
    const int v = lane >> 1, t = lane & 1;
    const int rr = v >> 2, rq = v & 3;
    const int rs = rr >> 1;
    const double *rd = wb + rr * kRowLen + rq * kQuarterOff + t * kPartials;
    // quarters rq = 0 (interior h0) and 1 (exterior h0) pass on the
    // whole-tile sums; 0 and 3 (exterior h1) store their own sums
    double *hdst_own = Ht + (rq == 0 ? 1 : 3) * C;
    const int pad0 = L & 1;             // zero channel after the m = 0 block
    const int n_pos = C + pad0;         // padded channel positions
    int slot = 0, base = 0;             // base: padded position of slot 0
    int xb = 0, xbase = 0;              // the exchange's batches, its first position
    // an exchange's lane: side io (0: interior, 1: exterior), entry xj; the
    // weights of the four tiles' sums in its in-group sum
    const bool x_on = lane < 2 * kXLen;
    const int io = (lane / kXLen) & 1, xj = lane & (kXLen - 1);
    double xw[kWavesPerBlock];
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; ++k) xw[k] = (io == 0 ? k < w : k > w) ? 1.0 : 0.0;
    const bool own_q = halves && tile_ok && t == 0 && (rq == 0 || rq == 3);
    auto exchange = [&]() {
        __syncthreads();
        const int pos = xbase + xj;
        double v[kWavesPerBlock];
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; ++k) v[k] = xch[k][io][xj];
        // interior: the tiles before this one; exterior: those after it (the
        // 0/1 weights make the FMAs plain sums)
        double sp = 0.0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; ++k) sp = fma(xw[k], v[k], sp);
        const int ch = pos < L ? pos : pos - pad0;
        if (x_on && tile_ok && pos < xbase + xb * 2 * kSlots && pos < n_pos &&
            !(pad0 && pos == L)) {
            Ht[2 * io * C + ch] = sp;
            if (io == 0 && w == kWavesPerBlock - 1) Gs[ch] = sp + v[kWavesPerBlock - 1];
            if (io == 1 && w == 0) Gs[C + ch] = sp + v[0];
        }
        __syncthreads();
        xbase += xb * 2 * kSlots;
        xb = 0;
    };
    auto flush = [&]() {
        wave_lds_sync();
        double acc = rd[0];
#pragma unroll
        for (int k = 1; k < kPartials; ++k) acc += rd[k];
        acc += dpp_quad<0xB1>(acc);
        const double whole = acc + dpp_row_shl4(acc);   // quarters 0, 1: + quarters 2, 3
        if (t == 0 && rq < 2) xch[w][rq][xb * 2 * kSlots + rr] = whole;
        const int pos = base + rr;      // padded position
        // padded position -> channel: the m = 0 block is positions 0..L-1
        const int ch = pos < L ? pos : pos - pad0;
        if (own_q && rs < slot && pos < n_pos && !(pad0 && pos == L))
            hdst_own[ch] = acc;
        wave_lds_sync();
        base += 2 * kSlots;
        slot = 0;
        if (++xb == kXBatches) exchange();
    };
    // one slot from two channels (R, I each)
    auto put2 = [&](double r0, double i0, double r1, double i1) {
        swap_rows16(r0, i0);
        swap_rows16(r1, i1);
        double *row = wr + slot * 2 * kRowLen;
        row[0] = r0 + i0;
        row[kRowLen] = r1 + i1;
        if (++slot == kSlots) flush();
    };

    // gamma_lm of the stream-order table, read one entry ahead of its use
    // through a running pointer (the read after the last entry lands on the
    // table's zero entry after the triangle; its value is never used)
    const double *ahead = reinterpret_cast<const double *>(tb.fq4 + 1);   // entry after the one held
    double ng = ld_const(reinterpret_cast<const double *>(tb.fq4), 0);   // the next entry to use
    auto next_gamma = [&]() {
        const double g = ng;
        ng = ld_const(ahead, 0);
        ahead += 4;
        return g;
    };
    // m = 0: channels l = 1..L (Qh_0^0 = 1 only seeds the recurrence; l = 0
    // is Gauss's law in the field kernel), two degrees per slot; the two Qh
    // registers trade roles instead of being copied
    {
        (void)next_gamma();                     // l = 0
        double Qa = 1.0, Qb = 0.0;              // Qh_{l-1}, Qh_{l-2}
        double sl = inv_r * inv_r2;             // r^-(2l+1) at l = 1
        int l = 1;
        for (; l < L; l += 2) {
            Qb = z * Qa - next_gamma() * r2 * Qb;   // Qh_l
            const double r0 = q * Qb, i0 = r0 * sl;
            sl *= inv_r2;
            Qa = z * Qb - next_gamma() * r2 * Qa;   // Qh_{l+1}
            const double r1 = q * Qa, i1 = r1 * sl;
            sl *= inv_r2;
            put2(r0, i0, r1, i1);
        }
        if (l == L) {
            Qb = z * Qa - next_gamma() * r2 * Qb;
            const double r0 = q * Qb;
            put2(r0, r0 * sl, 0.0, 0.0);
        }
    }
    if (FULL) {
        double Cm = 1.0, Sm = 0.0;
        double s_mm = inv_r;  // r^-(2m+1)
        for (int m = 1; m <= L; ++m) {
            const double nc = x * Cm - y * Sm;
            const double ns = x * Sm + y * Cm;
            Cm = nc;
            Sm = ns;
            s_mm *= inv_r2;
            const double qc = q * Cm, qs = q * Sm;
            double sl = s_mm;
            // cos and sin of one (l, m) fill one slot
            auto emit = [&](double Qv) {
                const double rc = Qv * qc, rs = Qv * qs;
                put2(rc, rc * sl, rs, rs * sl);
                sl *= inv_r2;
            };
            (void)next_gamma();                     // l = m: Qh_m^m = 1
            double Qa = 1.0, Qb = 0.0;
            emit(Qa);
            int l = m + 1;
            for (; l < L; l += 2) {
                Qb = z * Qa - next_gamma() * r2 * Qb;
                emit(Qb);
                Qa = z * Qb - next_gamma() * r2 * Qa;
                emit(Qa);
            }
            if (l == L) {
                Qb = z * Qa - next_gamma() * r2 * Qb;
                emit(Qb);
            }
        }
    }
    if (slot > 0) flush();   // last, partial batch: slots >= slot hold stale values
    if (xb > 0) exchange();
}

// ---------------------------------------------------------------------------
// Carries: prefix/suffix scans over groups, totals, coefficients, Q_diff
// ---------------------------------------------------------------------------

// The chunk's member and its group range; false if the member does not run.
__device__ inline bool chunk_groups(const Map &mp, const KParams &kp, int j, uint32_t *mb,
                                    int *g0, int *g1)
{
    const uint32_t m = mp.chunk_member[j];
    if (m == kNone || !member_runs(mp.seg[m], mp.ctl[m], kp)) return false;
    const Seg &sg = mp.seg[m];
    *mb = m;
    *g0 = (int)(sg.g0 + (uint32_t)(j - (int)sg.c0) * sg.cl);
    *g1 = min(*g0 + (int)sg.cl, (int)(sg.g0 + sg.ng));
    return true;
}

// A running FP64 sum that carries its own rounding error (Knuth's
// error-free TwoSum): the sum of n terms is good to about one rounding of
// the result instead of ~sqrt(n) of them.  The carries sum the group sums of
// up to ~6e4 groups per member; these kernels are bound by HBM, so the
// extra operations cost no time.
struct CompSum {
    double s = 0.0, e = 0.0;
    __device__ void add(double v)
    {
        const double t = s + v;
        const double z = t - s;
        e += (s - (t - z)) + (v - z);
        s = t;
    }
    __device__ double value() const { return s + e; }
};

// The group loops of the carry kernels issue the loads of kCarryBatch groups
// before using them (a chunk is 8-64 groups, or the tuned length, walked by
// one thread, and one HBM round trip per group would dominate); the sums
// keep the group order.
constexpr int kCarryBatch = 8;

__global__ __launch_bounds__(kBlock) void k_chunk_sums(Map mp, const double *__restrict__ GS,
                                                       double *__restrict__ chunkS, KParams kp)
{
    const int c = blockIdx.y * kBlock + threadIdx.x;
    if (c >= kp.SW) return;
    const int j = blockIdx.x;
    uint32_t mb;
    int g0, g1;
    if (!chunk_groups(mp, kp, j, &mb, &g0, &g1)) return;
    const size_t sw = (size_t)kp.SW;
    const double *src = GS + (size_t)g0 * sw + c;
    const int ng = g1 - g0;
    CompSum s;
    int g = 0;
    for (; g + kCarryBatch <= ng; g += kCarryBatch) {
        double v[kCarryBatch];
#pragma unroll
        for (int k = 0; k < kCarryBatch; ++k) v[k] = src[(size_t)(g + k) * sw];
#pragma unroll
        for (int k = 0; k < kCarryBatch; ++k) s.add(v[k]);
    }
    for (; g < ng; ++g) s.add(src[(size_t)g * sw]);
    chunkS[(size_t)j * kp.SW + c] = s.value();
}

// Per member (blockIdx.y) and channel (one wave each): exclusive prefix of the
// interior chunk sums and of the charge column, exclusive suffix of the
// exterior ones, and the totals T_lm.  The member's chunks, in scan order, are cut into 64 consecutive runs,
// one per lane: each lane sums its run, the wave scans the run sums, and each
// lane then writes its run's carries.
__global__ __launch_bounds__(kBlock) void k_chunk_scan(Map mp, const double *chunkS,
                                                       double *chunkC, double *T, KParams kp)
{
    const int lane = threadIdx.x & 63;
    const int c = (int)uniform_u32(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    const int s = blockIdx.y;
    if (c >= kp.SW) return;
    const Seg &sg = mp.seg[s];
    if (!member_runs(sg, mp.ctl[s], kp)) return;
    const int nc = (int)sg.nc;
    const bool interior = c < kp.C || c == kp.C2;
    const double *cS = chunkS + (size_t)sg.c0 * kp.SW + c;
    double *cC = chunkC + (size_t)sg.c0 * kp.SW + c;
    const int per = (nc + kWave - 1) / kWave;
    const int q0 = lane * per, q1 = min(q0 + per, nc);   // this lane's run in scan order
    auto chunk = [&](int q) { return interior ? q : nc - 1 - q; };
    CompSum part;
    for (int q = q0; q < q1; ++q) part.add(cS[(size_t)chunk(q) * kp.SW]);
    // inclusive scan of the runs' compensated sums (value and error term)
    CompSum incl = part;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double ts = __shfl_up(incl.s, o), te = __shfl_up(incl.e, o);
        if (lane >= o) {
            incl.add(ts);
            incl.e += te;
        }
    }
    CompSum run;
    run.s = __shfl_up(incl.s, 1);
    run.e = __shfl_up(incl.e, 1);
    if (lane == 0) run = CompSum();
    for (int q = q0; q < q1; ++q) {
        const size_t at = (size_t)chunk(q) * kp.SW;
        cC[at] = run.value();
        run.add(cS[at]);
    }
    if (!interior && lane == kWave - 1) T[(size_t)s * kp.C + (c - kp.C)] = incl.value();
}

// Per-group coefficients of the field kernel (FP64, absolute).  Interior
// coefficient of group g: the carry of the groups before it, plus the
// constant part: the image response -f_l T_lm and the hemisphere drive (odd
// l, m = 0; stream positions 0..L-1 hold m = 0, l = 1..L).  Exterior: the
// carry of the groups after it.  The field kernel adds the sums of the
// group's own tiles and halves.  Column C2: the charge of the member's
// particles before the group.  The block of the member's first chunk also
// records the probe response Q_diff(t_step) from the totals.
__global__ __launch_bounds__(kBlock) void k_chunk_apply(Map mp, const double *__restrict__ GS,
                                                        const double *__restrict__ chunkC,
                                                        const double *__restrict__ T, Tables tb,
                                                        KParams kp, double *__restrict__ CR,
                                                        double *__restrict__ qpre)
{
    const int c = blockIdx.y * kBlock + threadIdx.x;
    const int j = blockIdx.x;
    uint32_t mb;
    int g0, g1;
    if (!chunk_groups(mp, kp, j, &mb, &g0, &g1)) return;
    const Seg &sg = mp.seg[mb];
    const int64_t step = mp.ctl[mb].step;
    const bool in_run = step >= 0 && step < sg.n_steps;
    const double *Ts = T + (size_t)mb * kp.C;
    if (c == 0 && blockIdx.y == 0 && j == (int)sg.c0 && in_run) {
        double acc = 0.0;
        // m = 0 channel l sits at stream position l - 1; its total is a sum of Qh
        for (int l = 1; l <= kp.L; l += 2) acc += tb.drive_w[l] * tb.chn[l - 1] * Ts[l - 1];
        sg.qdiff[step] = -acc / sg.ntilde;
    }
    if (c >= kp.SW) return;
    const double inv_nt = sg.inv_ntilde;
    const size_t sw = (size_t)kp.SW;
    CompSum run;
    run.s = chunkC[(size_t)j * kp.SW + c];
    // Walks the chunk's groups in scan order (dir +1 from g0, -1 from g1 - 1),
    // calling f(g, carry before g) with the loads of kCarryBatch groups issued
    // ahead; the carry accumulates in group order, compensated.
    auto walk = [&](int dir, auto f) {
        const int ng = g1 - g0;
        const int first = dir > 0 ? g0 : g1 - 1;
        int i = 0;
        for (; i + kCarryBatch <= ng; i += kCarryBatch) {
            double v[kCarryBatch];
#pragma unroll
            for (int k = 0; k < kCarryBatch; ++k) v[k] = GS[(size_t)(first + dir * (i + k)) * sw + c];
#pragma unroll
            for (int k = 0; k < kCarryBatch; ++k) {
                f(first + dir * (i + k), run.value());
                run.add(v[k]);
            }
        }
        for (; i < ng; ++i) {
            const int g = first + dir * i;
            f(g, run.value());
            run.add(GS[(size_t)g * sw + c]);
        }
    };
    if (c == kp.C2) {   // charge of the member's particles before each group
        walk(1, [&](int g, double carry) { qpre[g] = carry; });
    } else if (c < kp.C) {
        const int l = tb.chl[c];
        const double nrm = tb.chn[c];
        const double w = tb.wl[l] * inv_nt * nrm;   // the sums are of Qh = Q / N_lm
        double k = -tb.ftil[l] * Ts[c] * w;
        if (c < kp.L && in_run) k += sg.u_asy[step] * tb.drive_w[l];
        walk(1, [&](int g, double carry) { CR[(size_t)g * kp.C2 + c] = (carry * w + k) * nrm; });
    } else {
        const int l = tb.chl[c - kp.C];
        const double nrm = tb.chn[c - kp.C];
        const double w = tb.wl[l] * inv_nt * nrm * nrm;   // sums of Qh; the field's Qh
        walk(-1, [&](int g, double carry) { CR[(size_t)g * kp.C2 + c] = carry * w; });
    }
}

// ---------------------------------------------------------------------------
// Counter-based generator for diffuse walls: Philox-4x64-10 (Salmon et al.,
// SC'11), counter (step, id, wall, 0), key (seed, 0).
// ---------------------------------------------------------------------------

__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Unit vector uniform on the hemisphere around the unit normal n.
__device__ inline void hemisphere_dir(uint64_t seed, uint32_t id, int64_t step, int wall,
                                      const double n[3], double d[3])
{
    uint64_t c[4] = {(uint64_t)step, (uint64_t)id, (uint64_t)wall, 0ull};
    philox4x64(c, seed, 0ull);
    const double inv53 = 1.0 / 9007199254740992.0;
    double ct = ((double)(c[0] >> 11) + 0.5) * inv53;
    double ph = 2.0 * kPi * (((double)(c[1] >> 11) + 0.5) * inv53);
    double st = sqrt(1.0 - ct * ct);
    double t[3] = {0.0, 0.0, 1.0};
    if (!(fabs(n[2]) < 0.9)) {
        t[0] = 1.0;
        t[2] = 0.0;
    }
    double ex[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2], t[0] * n[1] - t[1] * n[0]};
    double inv = 1.0 / sqrt(ex[0] * ex[0] + ex[1] * ex[1] + ex[2] * ex[2]);
    ex[0] *= inv;
    ex[1] *= inv;
    ex[2] *= inv;
    double ey[3] = {n[1] * ex[2] - n[2] * ex[1], n[2] * ex[0] - n[0] * ex[2],
                    n[0] * ex[1] - n[1] * ex[0]};
    double cp = cos(ph), sp = sin(ph);
    for (int j = 0; j < 3; ++j) d[j] = ct * n[j] + st * (cp * ex[j] + sp * ey[j]);
}

// ---------------------------------------------------------------------------
// Field and push
// ---------------------------------------------------------------------------

struct Grave {
    double *x, *y, *z, *vx, *vy, *vz;
    uint32_t *uid;
};

// Double-double values (hi + lo, |lo| <= ulp(hi) / 2) for the l = 0 field,
// where two fields of ~N^(1/2) times the result cancel: error-free products
// through the FMA and error-free sums (Knuth's TwoSum).
struct DD {
    double hi, lo;
};

__device__ inline DD dd_from_sum(double a, double b)
{
    const double s = a + b;
    const double z = s - a;
    return DD{s, (a - (s - z)) + (b - z)};
}

__device__ inline DD dd_add(DD a, DD b)
{
    const DD s = dd_from_sum(a.hi, b.hi);
    return dd_from_sum(s.hi, s.lo + (a.lo + b.lo));
}

__device__ inline DD dd_mul(DD a, double b)
{
    const double p = a.hi * b;
    const double e = fma(a.hi, b, -p);
    return dd_from_sum(p, fma(a.lo, b, e));
}

__device__ inline DD dd_div(DD a, DD b)
{
    const double q = a.hi / b.hi;
    // remainder a - q b, its leading part exact through the FMA
    const double r = (fma(-q, b.hi, a.hi) + a.lo) - q * b.lo;
    return dd_from_sum(q, r / b.hi);
}

__device__ inline DD dd_mul_dd(DD a, DD b)
{
    const double p = a.hi * b.hi;
    const double e = fma(a.hi, b.hi, -p);
    return dd_from_sum(p, e + (a.hi * b.lo + a.lo * b.hi));
}

// x*x + y*y + z*z in double-double: error-free squares, compensated sums.
__device__ inline DD dd_norm2(double x, double y, double z)
{
    const double xx = x * x, yy = y * y, zz = z * z;
    DD s = dd_add(DD{xx, fma(x, x, -xx)}, DD{yy, fma(y, y, -yy)});
    return dd_add(s, DD{zz, fma(z, z, -zz)});
}

// The l = 0 field (radial component) of the charge enclosed by radius r:
// the surface charge and the particles below, `charge` (exact), and the
// uniform ion background n_i: charge / (4 pi ntilde r^2) + n_i (r^3 - 1) / (3 r^2),
// formed in double-double from the position itself and rounded once.  The
// two terms are ~N^(1/2) times their sum at N particles, and taking r from
// the rounded radial key shifts both the same way for every particle near
// that radius: a few 1e-13 of the RMS field at 1.6e7 particles.
__device__ inline double gauss_field_uniform(double charge, double ntilde, double ion_density,
                                             double x, double y, double z)
{
    const DD r2 = dd_norm2(x, y, z);
    // r = sqrt(r2) to double-double: one Newton correction of the FP64 root
    const double rh = sqrt(r2.hi);
    const DD r{rh, (fma(-rh, rh, r2.hi) + r2.lo) / (2.0 * rh)};
    const DD r3 = dd_mul_dd(r, r2);
    const DD num2 = dd_mul(dd_add(r3, DD{-1.0, 0.0}), ion_density);
    const DD den2 = dd_mul(r2, 3.0);
    const DD four_pi{4.0 * 3.141592653589793116, 4.0 * 1.2246467991473532e-16};
    const DD den1 = dd_mul_dd(dd_mul(r2, ntilde), four_pi);
    const DD f = dd_add(dd_div(DD{charge, 0.0}, den1), dd_div(num2, den2));
    return f.hi + f.lo;
}

// Far field of all other tiles through this tile's coefficient vector
// (interior alpha then exterior beta, stream order), evaluated at scaled
// coordinates xi = x / rho in the working precision R; returns grad_xi Phi.
//   Phi(xi) = sum_lm Qh_l^m(z, r^2) U_lm,
//   U_lm = (beta + s_l alpha)^c C_m + (beta + s_l alpha)^s S_m,  s_l = r^-(2l+1),
//   V_lm = alpha^c C_m + alpha^s S_m,
// with the rescaled Qh_l^m = Q_l^m / N_lm (the coefficients carry N_lm):
// Qh_m^m = 1, Qh_l^m = z Qh_{l-1}^m - gamma_lm r^2 Qh_{l-2}^m, and D_z Qh its
// z-derivative at fixed r^2, D_z Qh_l = Qh_{l-1} + z D_z Qh_{l-1} - gamma r^2
// D_z Qh_{l-2}.  Qh_l^m C_m is homogeneous of degree l, so the radial
// derivative is exact by Euler's relation and only D_z Qh enters the
// tangential part:
//   grad Phi = rhat (1/r) sum [(l - m) Qh U - (2l+1) s_l Qh V]
//              + (e_z - cos th rhat) sum U D_z Qh + (sum Qh dU/dx, sum Qh dU/dy, 0).
// (Assembling the radial part from the two partial derivatives of Q instead
// loses a factor ~l to cancellation.)
// Where the far field reads the coefficients of channel k: interior and
// exterior side by side at p[2 (k - base)] and p[2 (k - base) + 1] (the
// channels of a few consecutive degrees lie within one LDS instruction's
// offset range of a single address).
template <typename R>
struct CfView {
    const R *p;
    int base;
    __device__ R a(int k) const { return p[2 * (k - base)]; }
    __device__ R b(int k) const { return p[2 * (k - base) + 1]; }
};

// stage(k0, k1) returns a view holding channels [k0, k1): the m = 0 block,
// then one m block at a time, in stream order.
//
// The coordinates come in FP64.  In FP32 (R = float) the far field is
// compensated: rounding the position to FP32 would shift every term of the
// recurrences coherently (a degree-l term by ~l ulps), and the terms of the
// tiles next to this one nearly cancel, which amplifies such shifts to
// ~1e-5 of the field.  So r^2 and z enter the Qh recurrence as hi + lo FP32
// pairs (the products with the lo parts are the first-order corrections,
// exact to O(ulp^2)), and the per-m quantities C_m, S_m, r^-(2m+1) and the
// directions are formed in FP64 and rounded once; what remains are the
// independent roundings of the FP32 arithmetic.
template <bool FULL, typename R, typename R4, typename Stage>
__device__ inline void far_field(Stage &&stage, int L, const R4 *fq, double xd, double yd,
                                 double zd, R &gx, R &gy, R &gz)
{
    constexpr bool kComp = sizeof(R) == 4;
    const double r2d = xd * xd + yd * yd + zd * zd;
    const double inv_r2d = 1.0 / r2d;
    const double inv_rd = kComp ? sqrt(inv_r2d) : 1.0 / sqrt(r2d);
    const R r2 = (R)r2d, z = (R)zd;
    const R r2l = kComp ? (R)(r2d - (double)r2) : (R)0;   // lo parts (zero in FP64)
    const R zl = kComp ? (R)(zd - (double)z) : (R)0;
    const R inv_r2 = (R)inv_r2d;
    // gamma r^2 and one step of the recurrences, with the lo corrections
    auto gam_r2 = [&](R g) -> R { return kComp ? fma(g, r2, g * r2l) : g * r2; };
    auto rec_q = [&](R Q1, R Q2, R gr2) -> R {
        return kComp ? fma(z, Q1, fma(zl, Q1, -gr2 * Q2)) : z * Q1 - gr2 * Q2;
    };
    auto rec_d = [&](R Q1, R D1, R D2, R gr2) -> R {
        return kComp ? fma(zl, D1, Q1 + z * D1) - gr2 * D2 : (Q1 + z * D1) - gr2 * D2;
    };
    R Ga = 0, Gz = 0, Gx = 0, Gy = 0;
    // With t_c = b_c + s_l a_c (s_l = r^-(2l+1)) each (l, m) adds to the radial
    // sum Qh [(l - m) t - (2l+1) s_l a] = (l - m) Qh b - (l + m + 1) s_l Qh a,
    // to the D_z sum Dz t and to the sum for d/dx, d/dy of C_m, S_m Qh t: each a
    // b part and an a part, two FMAs with the coefficient as scalar operand.
    // m = 0: cos channels only, stream position k = l - 1; l = 0 only seeds
    // the recurrence, its field is Gauss's law in the caller
    {
        R Q1 = 1, Q2 = 0, D1 = 0, D2 = 0;   // Qh_{l-1}, Qh_{l-2} and their D_z
        R sl = (R)(inv_rd * inv_r2d);       // r^-(2l+1) at l = 1
        const CfView<R> v = stage(0, L);
#pragma unroll 2
        for (int l = 1; l <= L; ++l) {
            const R4 e = fq[l];
            const R gr2 = gam_r2(e.x);
            const R Qv = rec_q(Q1, Q2, gr2);
            const R Dz = rec_d(Q1, D1, D2, gr2);
            const R ac = v.a(l - 1), bc = v.b(l - 1);
            const R Qs = Qv * sl, Qz = e.y * Qv, Qa = e.z * Qs, Ds = Dz * sl;
            Ga = fma(Qz, bc, Ga);
            Ga = fma(-Qa, ac, Ga);
            Gz = fma(Dz, bc, Gz);
            Gz = fma(Ds, ac, Gz);
            Q2 = Q1;
            Q1 = Qv;
            D2 = D1;
            D1 = Dz;
            sl *= inv_r2;
        }
    }
    if (FULL) {
        // C_m, S_m and C_{m-1}, S_{m-1} are common to all l of one m: the l
        // loop sums the cos and sin parts separately, combined once per m
        double Cmd = 1, Smd = 0, s_mmd = inv_rd;
        int j = L + 1;   // stream index of (m, l = m)
        int k = L;       // channel position of (m, l = m), cos then sin
        for (int m = 1; m <= L; ++m) {
            const R Cm1 = (R)Cmd, Sm1 = (R)Smd;
            {
                const double c1 = Cmd, s1 = Smd;
                Cmd = xd * c1 - yd * s1;
                Smd = xd * s1 + yd * c1;
            }
            s_mmd *= inv_r2d;
            const R Cm = (R)Cmd, Sm = (R)Smd;
            R sl = (R)s_mmd;
            // l = m: Qh = 1, D_z Qh = 0
            R Ac, As, Tc, Ts, Zc = 0, Zs = 0;
            const CfView<R> v = stage(k, k + 2 * (L - m + 1));
            {
                const R4 e = fq[j];
                const R ac = v.a(k), bc = v.b(k), as = v.a(k + 1), bs = v.b(k + 1);
                const R Qa = e.z * sl;
                Tc = sl * ac + bc;
                Ts = sl * as + bs;
                Ac = -Qa * ac;
                As = -Qa * as;
                ++j;
                k += 2;
                sl *= inv_r2;
            }
            R Q1 = 1, Q2 = 0, D1 = 0, D2 = 0;
#pragma unroll 2
            for (int l = m + 1; l <= L; ++l) {
                const R4 e = fq[j];
                const R ac = v.a(k), bc = v.b(k), as = v.a(k + 1), bs = v.b(k + 1);
                const R gr2 = gam_r2(e.x);
                const R Qv = rec_q(Q1, Q2, gr2);
                const R Dz = rec_d(Q1, D1, D2, gr2);
                const R Qs = Qv * sl, Qz = e.y * Qv, Qa = e.z * Qs, Ds = Dz * sl;
                Tc = fma(Qv, bc, Tc);
                Tc = fma(Qs, ac, Tc);
                Ts = fma(Qv, bs, Ts);
                Ts = fma(Qs, as, Ts);
                Zc = fma(Dz, bc, Zc);
                Zc = fma(Ds, ac, Zc);
                Zs = fma(Dz, bs, Zs);
                Zs = fma(Ds, as, Zs);
                Ac = fma(Qz, bc, Ac);
                Ac = fma(-Qa, ac, Ac);
                As = fma(Qz, bs, As);
                As = fma(-Qa, as, As);
                Q2 = Q1;
                Q1 = Qv;
                D2 = D1;
                D1 = Dz;
                ++j;
                k += 2;
                sl *= inv_r2;
            }
            const R dm = (R)m;
            Ga += Cm * Ac + Sm * As;
            Gz += Cm * Zc + Sm * Zs;
            Gx += dm * (Tc * Cm1 + Ts * Sm1);
            Gy += dm * (Ts * Cm1 - Tc * Sm1);
        }
    }
    const R inv_r = (R)inv_rd;
    const R xh = (R)(xd * inv_rd), yh = (R)(yd * inv_rd), c = (R)(zd * inv_rd);
    const R radial = Ga * inv_r - c * Gz;
    gx = xh * radial + Gx;
    gy = yh * radial + Gy;
    gz = c * Ga * inv_r + (xh * xh + yh * yh) * Gz;
}

// Near field: the direct part of G~_L between the particles of one block of
// W = 32 (a half tile) or 64 (the tile) radially consecutive particles (the
// pairs across blocks go through the coefficients), pair by pair.  For the pair (k, j) with
// rho = r_< / r_>, u = angular argument:
//   outer one: grad D = (1/r_>^2)       sum_l rho^l [-(l+1) P_l xh + P'_l v]
//   inner one: grad D = (1/(r_< r_>))   sum_l rho^l [ l P_l xh     + P'_l v]
// where v = xh_other - u xh (full) or e_z - cos(th) xh (axisymmetric).  The
// three sums are symmetric in (k, j), so each pair is evaluated once: at step
// s lane k takes partner k + s (mod W, inside its block) and hands the
// partner's gradient to it through a lane rotation.  Each term carries the
// charge of its source (the other particle of the pair).  Pair terms in R,
// accumulated in FP64.  The rows hold each block twice (entries h + i and
// h + i + W for the i-th particle of the block starting at entry h = 2 W b),
// so the partner of every shift is a plain offset.
template <bool FULL, typename R, typename NF>
__device__ inline void near_field(int lane, int W, int jn, int L, const NF *nf, const R *sxh,
                                  const R *syh, const R *szh, const R *sr, const R *sir,
                                  const R *sq, R xh, R yh, R zh, R r, R inv_r, R qk, double &ax,
                                  double &ay, double &az)
{
    const R inv_r2 = inv_r * inv_r;
    const int hl = lane & (W - 1), hb = 2 * (lane & W);
    for (int sft = 1; sft <= W / 2; ++sft) {
        const int jl = (lane & W) | ((hl + sft) & (W - 1));   // partner lane
        const int j = hb + hl + sft;
        const bool active = lane < jn && jl < jn && (sft < W / 2 || hl < W / 2);
        const R xj = sxh[j], yj = syh[j], zj = szh[j];
        const R rj = sr[j], irj = sir[j];
        const R qj = sq[j];
        // a block's lanes are in radial order (key (r^2, id)): the partner
        // is the inner one when it wraps below this lane
        const bool k_outer = hl + sft >= W;
        const R rho = k_outer ? rj * inv_r : r * irj;
        const R sc_out = k_outer ? inv_r2 : irj * irj;   // 1 / r_>^2
        const R sc_in = inv_r * irj;                     // 1 / (r_< r_>)
        const R u = FULL ? xh * xj + yh * yj + zh * zj : zh;
        R S1 = 0, Sl = 0, SBk = 0, SBj = 0;
        R P0 = 1, P1 = u, dP0 = 0, dP1 = 1;      // P_l(u) (own cos th if axisymmetric)
        R Q0 = 1, Q1 = zj, dQ0 = 0, dQ1 = 1;     // partner P_l(cos th_j), axisymmetric only
        R rl = rho;                              // l = 0 is Gauss's law in the caller
#pragma unroll 2
        for (int l = 1; l <= L; ++l) {
            const NF cl = nf[l];   // {(2l+1)/(l+1), l/(l+1), 2l+1, l}
            const R A = cl.x, Bc = cl.y, tl1 = cl.z, dl = cl.w;
            if (FULL) {
                const R t = rl * P1;
                S1 += t;
                Sl += dl * t;
                SBk += rl * dP1;
            } else {
                const R t = rl * P1 * Q1;
                S1 += t;
                Sl += dl * t;
                SBk += rl * dP1 * Q1;
                SBj += rl * P1 * dQ1;
                const R Q2 = A * zj * Q1 - Bc * Q0;
                const R dQ2 = dQ0 + tl1 * Q1;
                Q0 = Q1;
                Q1 = Q2;
                dQ0 = dQ1;
                dQ1 = dQ2;
            }
            const R P2 = A * u * P1 - Bc * P0;
            const R dP2 = dP0 + tl1 * P1;
            P0 = P1;
            P1 = P2;
            dP0 = dP1;
            dP1 = dP2;
            rl *= rho;
        }
        if (FULL) SBj = SBk;
        const R S_out = -(Sl + S1), S_in = Sl;
        const R SAk = k_outer ? S_out : S_in, sck = qj * (k_outer ? sc_out : sc_in);
        const R SAj = k_outer ? S_in : S_out, scj = qk * (k_outer ? sc_in : sc_out);
        R vkx, vky, vkz, vjx, vjy, vjz;
        if (FULL) {
            vkx = xj - u * xh; vky = yj - u * yh; vkz = zj - u * zh;
            vjx = xh - u * xj; vjy = yh - u * yj; vjz = zh - u * zj;
        } else {
            vkx = -zh * xh; vky = -zh * yh; vkz = 1 - zh * zh;
            vjx = -zj * xj; vjy = -zj * yj; vjz = 1 - zj * zj;
        }
        R gjx = scj * (SAj * xj + SBj * vjx);
        R gjy = scj * (SAj * yj + SBj * vjy);
        R gjz = scj * (SAj * zj + SBj * vjz);
        if (active) {
            ax += (double)(sck * (SAk * xh + SBk * vkx));
            ay += (double)(sck * (SAk * yh + SBk * vky));
            az += (double)(sck * (SAk * zh + SBk * vkz));
        } else {
            gjx = 0;
            gjy = 0;
            gjz = 0;
        }
        const int src = (lane & W) | ((hl - sft) & (W - 1));
        ax += (double)__shfl(gjx, src);
        ay += (double)__shfl(gjy, src);
        az += (double)__shfl(gjz, src);
    }
}

// One wave's particles for the near field: each block's rows written twice
// (see above).
template <typename R>
struct NearRows {
    R xh[2 * kWave], yh[2 * kWave], zh[2 * kWave], r[2 * kWave], ir[2 * kWave], q[2 * kWave];
    // FP32 only: r / rho_t - 1 against the tile's reference radius rho_t
    R s[sizeof(R) == 4 ? 2 * kWave : 1];
};

__device__ inline double bpermute(int addr, double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ inline float bpermute(int addr, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// Full near field.  Per pair (k, j), with rho = r_< / r_> and u = xh_k . xh_j:
//   S1 = sum_l rho^l P_l(u),  Sl = sum_l l rho^l P_l(u),  SB = sum_l rho^l P'_l(u)
// (l = 1..L) and, as above, S_in = Sl, S_out = -(Sl + S1).  For either particle
// the scale is 1 / (r_own r_>) whether it is the inner or the outer one, and
// grad D = (SA - SB u) xh_own + SB xh_other: a multiple of the own direction
// plus a multiple of the other's.  Each lane sums the multiples of its own
// direction in one number and the rest in a vector; the partner's two
// multiples go to it by a lane permutation, and it scales the sender's
// direction (read from LDS) itself.  Lanes without a particle carry charge 0,
// so their terms vanish without masks.  In FP64 the Legendre sums use the
// rescaled polynomials of the lg table (a two-operation recurrence; l = 1 is
// peeled); in FP32 a recurrence on P_l - P_{l-1} driven by 1 - u (lw table).
template <typename R, typename LG>
__device__ inline void near_field_full(int lane, int W, int L, const LG *lg, const NearRows<R> &nr,
                                       R xh, R yh, R zh, R r, R ir, R sk, R rho_t, R qk,
                                       double &ax, double &ay, double &az)
{
    double dck = 0.0, dbx = 0.0, dby = 0.0, dbz = 0.0;
    R ck = 0, bx = 0, by = 0, bz = 0;
    auto flush = [&]() {   // partial sums of a few shifts into FP64 (FP32 mode)
        dck += (double)ck;
        dbx += (double)bx;
        dby += (double)by;
        dbz += (double)bz;
        ck = 0;
        bx = 0;
        by = 0;
        bz = 0;
    };
    const LG c1 = lg[1];
    const int hl = lane & (W - 1), hb = 2 * (lane & W);
    auto shift = [&](const int sft, R qk_s, bool last) {
        const int j = hb + hl + sft;   // partner, in the doubled block row
        const R xj = nr.xh[j], yj = nr.yh[j], zj = nr.zh[j];
        const R rj = nr.r[j], irj = nr.ir[j];
        const R qj = last && hl >= W / 2 ? (R)0 : nr.q[j];
        // a block's lanes are in radial order (key (r^2, id)): the partner
        // hl + sft (mod W) is the inner one when it wraps below this lane
        const bool k_outer = hl + sft >= W;
        const R irmx = k_outer ? ir : irj;   // 1 / r_>
        R u, S1, Sl, SB;
        if constexpr (sizeof(R) == 4) {
            // rho = r_< / r_> = 1 - del with del = (s_> - s_<) rho_t / r_>
            // from the offsets s = r / rho_t - 1 (FP64-exact, small): del
            // keeps its relative precision, and the powers rho^l are stepped
            // as rl - rl del, so no rounding of rho (an absolute 2^-24 near
            // 1) is raised to the l-th power.
            const R del = fabsf(sk - nr.s[j]) * (rho_t * irmx);
            const R rho = 1.0f - del;
            // FP32: w = 1 - u = |xh_j - xh_k|^2 / 2 (for nearly parallel
            // directions the difference is exact, so w keeps its relative
            // precision where a dot product would leave 1 - u an absolute
            // 2^-24), and the Legendre recurrence runs on the scaled
            // differences E_l = l (P_l - P_{l-1}): E_{l+1} = E_l - (2l+1) w P_l,
            // P_{l+1} = P_l + E_{l+1} / (l+1).  Near u = 1, where the sums of
            // rho^l P_l and rho^l P'_l amplify errors in u, this keeps P_l to
            // FP32 relative precision.
            const R dx = xj - xh, dy = yj - yh, dz = zj - zh;
            const R w = 0.5f * fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            u = 1.0f - w;
            S1 = rho * u;
            Sl = S1;
            SB = rho;
            // two degrees per pass, the registers of degree l and l + 1
            // trading roles: (Pa, Da, dPa) hold P_l, E_l, P'_l and dPb
            // P'_{l-1}, which the first half overwrites with P'_{l+1}
            R Pa = u, Da = -w, dPa = 1, dPb = 0, rl = rho, Pb, Db;
            auto degree = [&](const LG c, R &P, R &D, R &dPm, R &Pn, R &Dn) {
                Dn = fmaf(-(c.z * w), P, D);
                Pn = fmaf(c.x, Dn, P);
                dPm = fmaf(c.z, P, dPm);   // P'_{l+1} = P'_{l-1} + (2l+1) P_l
                rl = fmaf(-rl, del, rl);
                const R t = rl * Pn;
                S1 += t;
                Sl = fmaf(c.w, t, Sl);
                SB = fmaf(rl, dPm, SB);
            };
            int l = 1;
            for (; l + 1 < L; l += 2) {
                degree(lg[l], Pa, Da, dPb, Pb, Db);       // degree l + 1
                degree(lg[l + 1], Pb, Db, dPa, Pa, Da);   // degree l + 2
            }
            if (l < L) degree(lg[l], Pa, Da, dPb, Pb, Db);
        } else {
            const R rmin = k_outer ? rj : r;   // r_<
            const R rho = rmin * irmx;
            u = xh * xj + yh * yj + zh * zj;
            // l = 1: P_1 = u, P'_1 = 1.  Then two degrees per pass with the
            // registers of Ph_l and Ph_{l-1} (and of P'_l, P'_{l-1}) trading
            // roles
            S1 = rho * u;
            Sl = S1;
            SB = rho;
            R Pa = u * u - c1.z, Pb = u, dPa = c1.w * u, dPb = 1, rl = rho * rho;
            int l = 2;
            for (; l < L; l += 2) {
                const LG ca = lg[l], cb = lg[l + 1];
                R t = rl * Pa;   // degree l from Pa
                S1 += ca.x * t;
                Sl += ca.y * t;
                SB += rl * dPa;
                Pb = u * Pa - ca.z * Pb;   // Ph_{l+1}
                dPb += ca.w * Pa;          // P'_{l+1}
                rl *= rho;
                t = rl * Pb;     // degree l + 1 from Pb
                S1 += cb.x * t;
                Sl += cb.y * t;
                SB += rl * dPb;
                Pa = u * Pb - cb.z * Pa;   // Ph_{l+2}
                dPa += cb.w * Pb;          // P'_{l+2}
                rl *= rho;
            }
            if (l == L) {
                const LG ca = lg[l];
                const R t = rl * Pa;
                S1 += ca.x * t;
                Sl += ca.y * t;
                SB += rl * dPa;
            }
        }
        const R S_out = -(Sl + S1), S_in = Sl;
        const R SAk = k_outer ? S_out : S_in, SAj = k_outer ? S_in : S_out;
        const R wk = qj * (ir * irmx), wj = qk_s * (irj * irmx);
        const R bk = wk * SB, bj = wj * SB;
        ck = fma(wk, SAk, ck);
        ck = fma(-bk, u, ck);
        bx = fma(bk, xj, bx);
        by = fma(bk, yj, by);
        bz = fma(bk, zj, bz);
        const R cj = fma(-bj, u, wj * SAj);
        // lane k's partner is k + sft (in its block), so lane k receives from
        // k - sft
        const int src_addr = 4 * ((lane & W) | ((hl - sft) & (W - 1)));
        const R cr = bpermute(src_addr, cj), br = bpermute(src_addr, bj);
        const int src = hb + hl + W - sft;   // in the doubled block row
        ck += cr;
        bx = fma(br, nr.xh[src], bx);
        by = fma(br, nr.yh[src], by);
        bz = fma(br, nr.zh[src], bz);
    };
    if constexpr (sizeof(R) == 4) {
        for (int s0 = 1; s0 < W / 2; s0 += 8) {
#pragma unroll 1
            for (int sft = s0; sft < min(s0 + 8, W / 2); ++sft) shift(sft, qk, false);
            flush();
        }
    } else {
#pragma unroll 1
        for (int sft = 1; sft < W / 2; ++sft) shift(sft, qk, false);
    }
    // the pairs (k, k + W/2) and (k + W/2, k) of a block are one pair: the
    // block's lanes below W/2 take it
    shift(W / 2, hl >= W / 2 ? (R)0 : qk, true);
    flush();
    ax += dck * (double)xh + dbx;
    ay += dck * (double)yh + dby;
    az += dck * (double)zh + dbz;
}

// FP32 (half the LDS rows, fewer registers) runs at six waves per SIMD;
// NEAR64: FP32 far field with the near field in FP64 (FP32 mode at high l_max)
template <bool FULL, bool FIELD_ONLY, bool FP32, bool NEAR64>
__global__ __launch_bounds__(kBlock, FP32 && !NEAR64 ? 6 : 4) void k_field_push(Map mp, State B, PRec *A, uint8_t *dead,
                                                       Grave G, const double *H,
                                                       const double *CR, const double *qpre,
                                                       Tables tb, KParams kp, double *Eout,
                                                       uint32_t *Eid, KeyRec *krec,
                                                       uint32_t *hist)
{
    // R, NF: the near field's precision; RF, NFF: the far field's
    using R = typename std::conditional<FP32 && !NEAR64, float, double>::type;
    using NF = typename std::conditional<FP32 && !NEAR64, float4, double4>::type;
    using RF = typename std::conditional<FP32, float, double>::type;
    using NFF = typename std::conditional<FP32, float4, double4>::type;
    // Per wave: the two halves' coefficients while the far field runs, then
    // the near field's rows.  The size keeps the block's LDS within a CU's
    // 160 KB at the kernel's occupancy (four blocks FP64, six FP32) and holds
    // a window of 288 FP64 channels (all of l_max 16) or 384 FP32 ones; the
    // second half's coefficients start kHalfPad bytes further, so that the two
    // addresses of a read fall on different banks.
    constexpr int kHalfPad = 16;
    constexpr int kLdsBytes = (FP32 && !NEAR64 ? 6144 : 9216) + kHalfPad;
    static_assert(sizeof(NearRows<R>) <= (size_t)kLdsBytes, "near-field rows exceed the wave's LDS");
    union WaveLds {
        NearRows<R> rows;
        RF cf[kLdsBytes / sizeof(RF)];
    };
    __shared__ WaveLds lds[kWavesPerBlock];

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const uint32_t group = blockIdx.x;
    const uint32_t tile = uniform_u32(group * kTilesPerGroup + w);
    // the tile's member: n = its alive count, pl = this lane's position in
    // its radial order
    uint32_t mb = kNone, n = 0, lt = 0;
    if ((int)tile < kp.n_tiles) {
        const uint32_t m = uniform_u32(mp.tile_member[tile]);
        if (m != kNone && member_runs(mp.seg[m], mp.ctl[m], kp)) {
            mb = m;
            n = mp.ctl[m].n_live;
            lt = tile - mp.seg[m].t0;
        }
    }
    const bool tile_live = mb != kNone && lt * kWave < n;
    const uint32_t p = tile * kWave + lane;
    const uint32_t pl = lt * kWave + lane;
    const bool valid = tile_live && pl < n;
    const int jn = tile_live ? (int)min((uint32_t)kWave, n - lt * kWave) : 0;

    // (the velocities are read at the push, so that they hold no registers
    // through the field evaluation)
    double x = 0.0, y = 0.0, z = 2.0;
    uint32_t uid = 0xffffffffu;
    if (valid) {
        x = B.x[p];
        y = B.y[p];
        z = B.z[p];
        uid = B.uid[p];
    }
    const double r2 = key_r2(x, y, z);
    const double r = sqrt(r2);
    const double inv_r = 1.0 / r;
    const double inv_r2 = 1.0 / r2;
    const double xh = x * inv_r, yh = y * inv_r, zh = z * inv_r;
    const bool ion = valid && (uid & kIonBit);
    const double qk = ion ? 1.0 : kQ;   // this particle's charge
    if (!tile_live) return;

    const int L = kp.L;
    const Seg &sg = mp.seg[mb];
    Ctl &ct = mp.ctl[mb];
    const double ntilde = sg.ntilde, inv_nt = sg.inv_ntilde;
    // the rows of the group's tiles (half sums, half charges)
    const double *Hg = H + (size_t)group * kTilesPerGroup * kp.HW;
    // the near field's block: a half tile (the halves' coefficients differ by
    // the other half's sums) or the whole tile (they are the same)
    const int NW = (int)uniform_u32((uint32_t)sg.near_w);
    const bool split = NW == kHalf;

    // FP32: the tile's reference radius rho_t, its first particle's (the far
    // field's coordinates and coefficients are scaled by it; the near field
    // measures radii from it).
    double rho = 1.0;
    if (FP32) {
        const uint32_t p0 = tile * kWave;
        rho = sqrt(key_r2(B.x[p0], B.y[p0], B.z[p0]));
    }
    const double inv_rho = 1.0 / rho;

    // ---- far field (all particles outside this lane's near-field block) ----
    double Ex, Ey, Ez;
    {
        RF gx, gy, gz;
        const NFF *fq;
        if constexpr (FP32) fq = tb.fq4_32;
        else fq = tb.fq4;
        const double xs = x * inv_rho, ys = y * inv_rho, zs = z * inv_rho;
        // Coefficients of channel c for half h of this tile: the group's
        // (carries of the groups before and after it, the image response and
        // the drive) plus the sums of the group's own particles on each side:
        //   interior: the tiles before this one, and for h = 1 half 0;
        //   exterior: the tiles after this one, and for h = 0 half 1;
        // (the halves' own terms only with a near field per half tile)
        // as raw sums of Qh times N_lm^2 / ((2l+1) ntilde).  FP32: scaled to
        // the tile's coordinates x / rho (interior rho^-(l+1), exterior
        // rho^l) in FP64, then rounded once.  Every pass of every lane reads
        // them, so they go to LDS (the far field reads them as broadcasts, one
        // address per half), in windows of kWin channels (interior and
        // exterior of both halves) that hold whole m blocks; a window moves on
        // when the next block does not fit (never at l_max <= 16).  An m block
        // has at most 2 l_max <= 128 channels.
        constexpr int kWin = (kLdsBytes - kHalfPad) / (int)sizeof(RF) / 4;
        constexpr int kH1 = 2 * kWin + kHalfPad / (int)sizeof(RF);   // half 1's offset
        static_assert(kWin >= 2 * kMaxL, "an m block must fit a window");
        RF *cbuf = reinterpret_cast<RF *>(lds[w].cf);
        const int C = kp.C;
        const double *CRg = CR + (size_t)group * kp.C2;
        // FP32: rho^-(l+1) and rho^l of degree l = lane + 1, fetched per
        // channel from the lane of its degree
        double pw_in = 1.0, pw_out = 1.0;
        if (FP32) {
            const double lg = log2(rho);
            pw_in = exp2(-(lane + 2.0) * lg);
            pw_out = exp2((lane + 1.0) * lg);
        }
        int win0 = 0, win_len = -1;   // resident channels [win0, win0 + win_len)
        // Fills the window with channels [k0, k0 + len), U channels per lane at a
        // time with all their loads issued before the first use.  The first
        // window is filled before the far field starts (no other work of the
        // wave could hide its loads then, and few registers are live: U = 2);
        // a window moved inside the far field fills two channels at a time at
        // four waves per SIMD, one at six.
        auto fill = [&](int k0, int len, auto u_tag) {
            constexpr int U = decltype(u_tag)::value;
            const int n_iter = (len + kWave - 1) / kWave;
            for (int it0 = 0; it0 < n_iter; it0 += U) {
                double yin[U], yout[U], hin[U], hout[U], ci[U], co[U], gsc[U];
                int src[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = (it0 + u) * kWave + lane;
                    const int c = k0 + (i < len ? i : 0);
                    // the interior sums of the group's tiles before this one,
                    // the exterior sums of those after it, and the halves' own
                    // sums
                    const double *Ht = Hg + w * kp.HW;
                    yin[u] = Ht[c];
                    yout[u] = Ht[2 * C + c];
                    hin[u] = split ? Ht[C + c] : 0.0;
                    hout[u] = split ? Ht[3 * C + c] : 0.0;
                    ci[u] = CRg[c];
                    co[u] = CRg[C + c];
                    gsc[u] = tb.chg[c] * inv_nt;
                    src[u] = FP32 ? 4 * (tb.chl[c] - 1) : 0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = (it0 + u) * kWave + lane;
                    double a0 = ci[u] + gsc[u] * yin[u], a1 = ci[u] + gsc[u] * (yin[u] + hin[u]);
                    double b1 = co[u] + gsc[u] * yout[u], b0 = co[u] + gsc[u] * (yout[u] + hout[u]);
                    if (FP32) {
                        // every lane takes part in the fetches
                        const double si = bpermute(src[u], pw_in), so = bpermute(src[u], pw_out);
                        a0 *= si;
                        a1 *= si;
                        b0 *= so;
                        b1 *= so;
                    }
                    if (i < len) {
                        cbuf[2 * i] = (RF)a0;
                        cbuf[2 * i + 1] = (RF)b0;
                        cbuf[kH1 + 2 * i] = (RF)a1;
                        cbuf[kH1 + 2 * i + 1] = (RF)b1;
                    }
                }
            }
            wave_lds_sync();
            win0 = k0;
            win_len = len;
        };
        fill(0, min(kWin, C), std::integral_constant<int, 2>());
        auto stage = [&](int k0, int k1) {
            if (k1 > win0 + win_len) {
                wave_lds_sync();   // the old window's reads are done
                // (the FP32 kernel at six waves per SIMD has no registers to spare)
                fill(k0, min(kWin, C - k0), std::integral_constant<int, FP32 && !NEAR64 ? 1 : 2>());
            }
            return CfView<RF>{cbuf + (lane >= kHalf ? kH1 : 0), win0};
        };
        far_field<FULL, RF>(stage, L, fq, xs, ys, zs, gx, gy, gz);
        wave_lds_sync();   // read before the rows below overwrite them
        Ex = -(double)gx * inv_rho;
        Ey = -(double)gy * inv_rho;
        Ez = -(double)gz * inv_rho;
    }

    // ---- near field (own block); E += -(1 / (4 pi nt)) sum_j q_j grad D ----
    NearRows<R> &nr = lds[w].rows;
    {
        const int e0 = 2 * (lane & NW) + (lane & (NW - 1));   // entries e0, e0 + NW
        for (int c = 0; c < 2; ++c) {
            const int i = e0 + c * NW;
            nr.xh[i] = (R)xh;
            nr.yh[i] = (R)yh;
            nr.zh[i] = (R)zh;
            nr.r[i] = (R)r;
            nr.ir[i] = (R)inv_r;
            nr.q[i] = valid ? (R)qk : (R)0;
            if constexpr (sizeof(R) == 4) nr.s[i] = (R)(r * inv_rho - 1.0);
        }
    }
    wave_lds_sync();   // the rows are this wave's own
    {
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (L < 1) {
            // monopole only: Gauss's law below
        } else if constexpr (FULL) {
            const NF *lg;
            if constexpr (std::is_same<R, float>::value) lg = tb.lw4_32;
            else lg = tb.lg4;
            near_field_full<R, NF>(lane, NW, L, lg, nr, (R)xh, (R)yh, (R)zh, (R)r, (R)inv_r,
                                   (R)(r * inv_rho - 1.0), (R)rho, valid ? (R)qk : (R)0, ax,
                                   ay, az);
        } else {
            const NF *nf;
            if constexpr (std::is_same<R, float>::value) nf = tb.nf4_32;
            else nf = tb.nf4;
            near_field<FULL, R, NF>(lane, NW, jn, L, nf, nr.xh, nr.yh, nr.zh, nr.r, nr.ir, nr.q,
                                    (R)xh, (R)yh, (R)zh, (R)r, (R)inv_r, (R)qk, ax, ay, az);
        }
        const double cn = -1.0 / (4.0 * kPi * ntilde);
        Ex += cn * ax;
        Ey += cn * ay;
        Ez += cn * az;
    }

    // ---- self-image correction: the totals T_lm include the particle's own
    // image, which the pair sum i != k excludes ----
    {
        double sr = 0.0, sz = 0.0;   // radial and (e_z - c xh) parts of grad Phi_self
        double rl = inv_r2 * inv_r2 * inv_r;   // r^-(2l+3) at l = 1
        if (FULL) {
            for (int l = 1; l <= L; ++l) {
                sr += tb.self_w[l] * (l + 1.0) * rl;
                rl *= inv_r2;
            }
            // grad Phi_self = -q sum f_l (l+1)/(4 pi nt) r^-(2l+3) xh; E = -grad
            const double e = qk * inv_nt * sr;
            Ex += e * xh;
            Ey += e * yh;
            Ez += e * zh;
        } else {
            double P0 = 1.0, P1 = zh, dP0 = 0.0, dP1 = 1.0;
            for (int l = 1; l <= L; ++l) {
                sr += tb.self_w[l] * rl * P1 * (-(l + 1.0) * P1);
                sz += tb.self_w[l] * rl * P1 * dP1;
                const double P2 = tb.nfA[l] * zh * P1 - tb.nfB[l] * P0;
                const double dP2 = dP0 + (2.0 * l + 1.0) * P1;
                P0 = P1;
                P1 = P2;
                dP0 = dP1;
                dP1 = dP2;
                rl *= inv_r2;
            }
            // grad Phi_selfcorr = q sum (f_l/(4 pi nt)) r^-(2l+3) P_l [-(l+1) P_l xh + P'_l (e_z - c xh)]
            const double qn = qk * inv_nt;
            const double gx = qn * (sr * xh + sz * (-zh * xh));
            const double gy = qn * (sr * yh + sz * (-zh * yh));
            const double gz = qn * (sr * zh + sz * (1.0 - zh * zh));
            Ex -= gx;
            Ey -= gy;
            Ez -= gz;
        }
    }

    // ---- l = 0: Gauss's law.  The l = 0 part of G~ is 1/(4 pi r_>), so only
    // the charge enclosed by r_k pushes: Q_S, the particles before k in the
    // radial order (those of earlier tiles, carried by the scan, and the
    // lanes below in this tile), exact counts in super-particle units, and
    // the immobile ion background.  The particles' and the uniform
    // background's fields nearly cancel (to ~N^-1/2 of each), so they are
    // formed and added in double-double; a profile's enclosed charge is
    // tabulated and joins the count. ----
    {
        const uint64_t below = (1ull << lane) - 1ull;
        const int n_below = __popcll(__ballot(valid) & below);
        const int i_below = __popcll(__ballot(ion) & below);
        // the group's particles before this tile (exact counts)
        const double in_group = Hg[w * kp.HW + 4 * kp.C];
        const double before =
            (qpre[group] + in_group) + ((double)i_below + kQ * (double)(n_below - i_below));
        double e;
        if (sg.ion_tab) {
            e = ((ct.q_surface + before) + ion_enclosed(sg, r, r2)) / (4.0 * kPi * ntilde * r2);
        } else if constexpr (FP32) {
            // FP64 rounding of the two opposing terms leaves ~1e-16 sqrt(N) of
            // the field, far below the FP32 mode's error
            const double q_enc = ct.q_surface + before;
            e = (q_enc / (4.0 * kPi * ntilde) + sg.ion_density * (r2 * r - 1.0) / 3.0) * inv_r2;
        } else {
            e = gauss_field_uniform(ct.q_surface + before, ntilde, sg.ion_density, x, y, z);
        }
        Ex += e * xh;
        Ey += e * yh;
        Ez += e * zh;
    }

    if (FIELD_ONLY) {
        if (valid) {
            Eout[3 * (size_t)p + 0] = Ex;
            Eout[3 * (size_t)p + 1] = Ey;
            Eout[3 * (size_t)p + 2] = Ez;
            Eid[p] = uid;
        }
        return;
    }
    if (!valid) return;

    // ---- leapfrog (Sec. 4 equations of motion) ----
    const double qm = ion ? sg.ion_qm : kQ / kM;
    const double dt = sg.dt;
    double vx = B.vx[p], vy = B.vy[p], vz = B.vz[p];
    vx = __dadd_rn(vx, __dmul_rn(qm * Ex, dt));
    vy = __dadd_rn(vy, __dmul_rn(qm * Ey, dt));
    vz = __dadd_rn(vz, __dmul_rn(qm * Ez, dt));
    x = __dadd_rn(x, __dmul_rn(vx, dt));
    y = __dadd_rn(y, __dmul_rn(vy, dt));
    z = __dadd_rn(z, __dmul_rn(vz, dt));

    // ---- walls (tested on the new position) ----
    const double rn = sqrt(key_r2(x, y, z));
    uint8_t absorbed = 0;
    const int64_t step = ct.step;
    const double r_out = sg.r_out;
    if (rn <= 1.0 || rn >= r_out) {
        const bool probe = rn <= 1.0;
        const int bc = probe ? sg.probe_bc : sg.wall_bc;
        if (probe && bc == SIM_BC_ABSORB) {
            absorbed = 1;
        } else {
            const double s = probe ? (2.0 - rn) / rn : (2.0 * r_out - rn) / rn;
            const double nrm[3] = {x / rn, y / rn, z / rn};
            x = x * s;
            y = y * s;
            z = z * s;
            if (bc == SIM_BC_DIFFUSE) {
                const double sp = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(vx, vx), __dmul_rn(vy, vy)),
                                                 __dmul_rn(vz, vz)));
                double inw[3] = {nrm[0], nrm[1], nrm[2]};
                if (!probe) {
                    inw[0] = -inw[0];
                    inw[1] = -inw[1];
                    inw[2] = -inw[2];
                }
                double d[3];
                hemisphere_dir(sg.seed, uid, step, probe ? 0 : 1, inw, d);
                vx = sp * d[0];
                vy = sp * d[1];
                vz = sp * d[2];
            } else {
                const double vn = __dadd_rn(__dadd_rn(__dmul_rn(vx, nrm[0]), __dmul_rn(vy, nrm[1])),
                                            __dmul_rn(vz, nrm[2]));
                const double two_vn = 2.0 * vn;
                vx = __dsub_rn(vx, __dmul_rn(two_vn, nrm[0]));
                vy = __dsub_rn(vy, __dmul_rn(two_vn, nrm[1]));
                vz = __dsub_rn(vz, __dmul_rn(two_vn, nrm[2]));
            }
        }
    }
    PRec out;
    out.x = x;
    out.y = y;
    out.z = z;
    out.vx = vx;
    out.vy = vy;
    out.vz = vz;
    out.uid = uid;
    out.pad[0] = out.pad[1] = out.pad[2] = 0u;
    A[p] = out;
    dead[p] = absorbed;
    // the next step's sort record of this slot, when the member runs then
    // (the same key, bucket and atomic slot as the key kernel would take;
    // the histogram was cleared by this step's offsets kernel)
    if (kp.fuse_keys && step + 1 < sg.n_steps) {
        KeyRec kr{0ull, 0u, kNone};
        if (!absorbed) {
            const double k2 = key_r2(x, y, z);
            kr.key = (uint64_t)__double_as_longlong(k2);
            kr.uid = uid;
            kr.sub = atomicAdd(&hist[bucket_of(k2, sg.inv_vol, sg.b0, sg.nb)], 1u);
        }
        krec[p] = kr;
    }
    if (absorbed) {
        if (ion) atomicAdd(&ct.n_dead_ion, 1u);
        const uint32_t slot = sg.p0 + atomicAdd(&ct.n_dead, 1u);
        G.x[slot] = x;
        G.y[slot] = y;
        G.z[slot] = z;
        G.vx[slot] = vx;
        G.vy[slot] = vy;
        G.vz[slot] = vz;
        G.uid[slot] = uid;
    }
}

__global__ void k_step_finish(Map mp, KParams kp)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= kp.n_members) return;
    Ctl &c = mp.ctl[s];
    const Seg &sg = mp.seg[s];
    if (!member_runs(sg, c, kp)) return;
    c.step += 1;
    c.n_cur = c.n_live;
    // the push produced the sort records of the step the member runs next
    if (kp.fuse_keys && c.step < sg.n_steps) c.keys_for = c.step;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

enum KernelId {
    KN_SORT_KEY, KN_SCAN_A, KN_SCAN_C, KN_SORT_SCATTER, KN_SORT_RANK, KN_MOMENTS,
    KN_CHUNK_SUMS, KN_CHUNK_SCAN, KN_CHUNK_APPLY, KN_FIELD_PUSH, KN_STEP_FINISH, KN_COUNT
};

const char *kKernelNames[KN_COUNT] = {
    "sort_key", "bucket_sums", "bucket_offsets", "sort_scatter",
    "sort_rank_move", "moments", "carry_chunk_sums", "carry_chunk_scan", "carry_apply",
    "field_push", "step_finish"};

// What all members of a handle share, and the handle's capacities.
// The tunable launch sizes of sim_params, with 0 resolved to the built-in
// choice (bucket) or kept as "automatic" (chunk).
struct Tuning {
    int bucket = kBucketOccupancy;   // mean particles per sort bucket
    int chunk = 0;                   // groups per carry chunk, 0: by member size
    int keys = 0;                    // sort keys: 1 push, -1 own pass, 0 by extent
    int split = 0;                   // near field: 1 half tiles, -1 whole tiles, 0 by member
};

Tuning tuning_of(const sim_params *p)
{
    Tuning t;
    if (p->sort_bucket > 0) t.bucket = p->sort_bucket;
    if (p->carry_chunk > 0) t.chunk = p->carry_chunk;
    t.keys = p->sort_keys;
    t.split = p->near_split;
    return t;
}

// Particles of a member's near-field block.  Half tiles halve the pair sums;
// the pairs across the halves then go through the coefficients.  In FP32 the
// coefficients carry the force of a close pair to a few ulps times l_max,
// while the pair's force is about l_max^2 / sqrt(n) of the RMS field (the
// collective field of n particles grows as sqrt(n)): half tiles are used
// where l_max^2 <= sqrt(n).  FP64 always splits.
int near_width(const Tuning &tu, bool fp32, int L, int64_t n)
{
    if (tu.split != 0) return tu.split > 0 ? kHalf : kWave;
    if (!fp32) return kHalf;
    return (double)L * (double)L <= std::sqrt((double)n) ? kHalf : kWave;
}

// In the FP32 mode the near field's FP32 error grows with l_max: a pair at
// nearly equal radius and angle contributes up to ~l_max^2 / (4 pi ntilde r^2)
// to the field, many times the field's RMS when the tile is sparse, and the
// FP32 evaluation of such a pair carries a few ulps of it.  With the radial
// powers stepped from 1 - rho and the Legendre recurrence driven by 1 - u it
// stays near 2-5e-6 of the RMS field up to l_max 19 on random shells of a few
// thousand particles; from this degree on the near field runs in FP64 while
// the far field stays FP32 (compensated).
constexpr int kNear64MinL = 20;

struct Layout {
    int L, C, C2;
    bool full, fp32;
    bool near64;     // FP32 mode with an FP64 near field (l_max >= kNear64MinL)
    int n_tiles;     // particle slots / 64 (whole groups)
    int n_groups;    // n_tiles / 4
    int n_chunks;
    int nb, nb_blocks;
    int n_members;
    Tuning tu;
};

// The part of the capacities in use: every member's tiles, chunks, buckets
// and table index lie below these (at least 1 each).  Launch grids cover the
// extent, not the capacity, so a large, sparsely filled handle steps at the
// cost of what it holds.
struct Extent {
    int n_tiles = kTilesPerGroup, n_chunks = 1, nb = 1, nb_blocks = 1, n_members = 1;
    bool operator==(const Extent &o) const
    {
        return n_tiles == o.n_tiles && n_chunks == o.n_chunks && nb == o.nb &&
               n_members == o.n_members;
    }
};

// Per-member sizes: groups, tiles (4 per group), chunks, buckets, groups per chunk.
struct MemberShape {
    uint32_t ng, nt, nc, nb, cl;
};

uint32_t groups_for(int64_t n) { return (uint32_t)((n + kGroupSlots - 1) / kGroupSlots); }

MemberShape member_shape(int64_t n, const Tuning &tu)
{
    MemberShape m;
    m.ng = groups_for(n);
    m.nt = m.ng * kTilesPerGroup;
    if (tu.chunk > 0) {
        m.cl = (uint32_t)tu.chunk;
    } else {
        m.cl = kChunkMin;
        while (m.cl < (uint32_t)kChunkMax && (uint64_t)m.cl * kChunkTarget < m.ng) m.cl *= 2;
    }
    m.nc = (m.ng + m.cl - 1) / m.cl;
    m.nb = (uint32_t)std::max<int64_t>(1, n / tu.bucket);
    return m;
}

bool check_common(const sim_params *p, std::string *why)
{
    if (!p) { *why = "params is NULL"; return false; }
    if (p->struct_size != sizeof(sim_params)) { *why = "params struct_size mismatch"; return false; }
    if (p->l_max < 0 || p->l_max > kMaxL) { *why = "l_max must be in [0, 64]"; return false; }
    if (!(p->d > 0.0 && p->d < 1.0)) { *why = "d must be in (0, 1)"; return false; }
    if (!(p->eps_r > 0.0) || !std::isfinite(p->eps_r)) { *why = "eps_r must be > 0"; return false; }
    if (p->m_mode != SIM_M_FULL && p->m_mode != SIM_M_AXISYM) { *why = "bad m_mode"; return false; }
    if (p->precision != SIM_FP64 && p->precision != SIM_FP32_COMP) { *why = "bad precision"; return false; }
    if (p->tile != 0 && p->tile != kWave) { *why = "tile must be 0 or 64"; return false; }
    if (p->sort_bucket < 0 || p->sort_bucket > 256) { *why = "sort_bucket must be 0 or in [1, 256]"; return false; }
    if (p->sort_keys < -1 || p->sort_keys > 1) { *why = "sort_keys must be -1, 0 or 1"; return false; }
    if (p->near_split < -1 || p->near_split > 1) { *why = "near_split must be -1, 0 or 1"; return false; }
    if (p->carry_chunk != 0 && (p->carry_chunk < kChunkMin || p->carry_chunk > 1024)) {
        *why = "carry_chunk must be 0 or in [8, 1024]";
        return false;
    }
    return true;
}

// Scalar checks of a member (the particle arrays are checked at admission).
bool check_member_scalars(const sim_member *m, std::string *why)
{
    if (!m) { *why = "member is NULL"; return false; }
    if (m->struct_size != sizeof(sim_member)) { *why = "member struct_size mismatch"; return false; }
    if (m->n <= 0 || m->n > 0x7fffffffLL) { *why = "n must be in [1, 2^31)"; return false; }
    if (m->n_steps < 0) { *why = "n_steps < 0"; return false; }
    if (m->start_step < 0 || m->start_step > m->n_steps) {
        *why = "start_step outside [0, n_steps]";
        return false;
    }
    if (!(m->r_out > 1.0) || !std::isfinite(m->r_out)) { *why = "r_out must be > 1"; return false; }
    if (!(m->dt > 0.0) || !std::isfinite(m->dt)) { *why = "dt must be > 0"; return false; }
    if (!(m->ntilde > 0.0) || !std::isfinite(m->ntilde)) { *why = "ntilde must be > 0"; return false; }
    if (!(m->ion_density >= 0.0) || !std::isfinite(m->ion_density)) {
        *why = "ion_density must be >= 0";
        return false;
    }
    if (!std::isfinite(m->q_surface0)) { *why = "q_surface0 must be finite"; return false; }
    if (!(m->ion_mass >= 0.0) || !std::isfinite(m->ion_mass)) { *why = "ion_mass must be >= 0"; return false; }
    if (m->ion_profile && (m->ion_profile_len < 2 || m->ion_profile_len > (1 << 24))) {
        *why = "ion_profile_len must be in [2, 2^24]";
        return false;
    }
    if (m->probe_bc < SIM_BC_ABSORB || m->probe_bc > SIM_BC_DIFFUSE) { *why = "bad probe_bc"; return false; }
    if (m->wall_bc != SIM_BC_SPECULAR && m->wall_bc != SIM_BC_DIFFUSE) { *why = "bad wall_bc"; return false; }
    return true;
}

// chunks < 0: room for any mix of members (every tile in the shortest
// chunks, plus one partial chunk per member); else exactly that many.
bool make_layout(const sim_params *p, int64_t slots, int32_t max_members, int64_t chunks,
                 Layout *lo, std::string *why)
{
    if (!check_common(p, why)) return false;
    if (slots <= 0 || slots > 0x7fffffffLL - kGroupSlots) { *why = "slot capacity must be in [1, 2^31 - 256)"; return false; }
    if (max_members <= 0 || max_members > (1 << 20)) { *why = "max_members must be in [1, 2^20]"; return false; }
    lo->L = p->l_max;
    lo->full = p->m_mode == SIM_M_FULL;
    lo->fp32 = p->precision == SIM_FP32_COMP;
    lo->near64 = lo->fp32 && p->l_max >= kNear64MinL;
    lo->C = lo->full ? (p->l_max + 1) * (p->l_max + 1) - 1 : p->l_max;
    lo->C2 = 2 * lo->C;
    lo->n_groups = (int)groups_for(slots);
    lo->n_tiles = lo->n_groups * kTilesPerGroup;
    lo->n_members = max_members;
    lo->tu = tuning_of(p);
    // every member rounds its chunks and buckets up by at most one
    const int cl_min = lo->tu.chunk > 0 ? lo->tu.chunk : kChunkMin;
    lo->n_chunks = chunks >= 0 ? (int)std::max<int64_t>(1, chunks)
                               : (lo->n_groups + cl_min - 1) / cl_min + max_members;
    lo->nb = (int)std::max<int64_t>(1, slots / lo->tu.bucket) + (max_members > 1 ? max_members : 0);
    lo->nb_blocks = (lo->nb + kScanPerBlock - 1) / kScanPerBlock;
    return true;
}

struct Alloc {
    std::vector<std::pair<void **, size_t>> items;
    template <class T> void add(T **ptr, size_t count) { items.push_back({(void **)ptr, count * sizeof(T)}); }
    size_t total() const {
        size_t s = 0;
        for (auto &it : items) s += (it.second + 255) & ~size_t(255);
        return s;
    }
};

// Bytes of a member's arrays in the batch's data pool: drive and response
// (8 B per step each) and, with an ion profile of prof_len nodes, its node
// densities and enclosed charges (16 B per node), each 256-byte aligned.
constexpr size_t kPoolUnit = 256;

size_t align_unit(size_t b) { return (b + kPoolUnit - 1) & ~(kPoolUnit - 1); }

size_t member_bytes(int64_t n_steps, int64_t prof_len)
{
    return 2 * align_unit((size_t)std::max<int64_t>(n_steps, 1) * 8) +
           (prof_len > 0 ? align_unit((size_t)prof_len * 16) : 0);
}

// First-fit allocator of ranges [start, start + len) of a capacity.
class Ranges {
public:
    void reset(uint32_t capacity)
    {
        free_.clear();
        if (capacity) free_[0] = capacity;
    }
    bool take(uint32_t len, uint32_t *start)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *start = it->first;
                const uint32_t rest = it->second - len, at = it->first + len;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void give(uint32_t start, uint32_t len)
    {
        auto it = free_.emplace(start, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<uint32_t, uint32_t> free_;
};

struct Member {
    bool used = false;
    Seg seg{};
    uint32_t md_start = 0, md_units = 0;   // the member's range of the data pool
    int64_t n = 0;
    int64_t step_host = 0;    // absolute step after all enqueued work
    int64_t start_step = 0;
    double q_surface0 = 0.0;
    std::vector<std::pair<uint32_t, int64_t>> id_index;  // (uid, creation index), sorted
};

}  // namespace

struct sim {
    sim_params prm;
    Layout lo;
    Extent ext;
    KParams kp;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    PRec *A = nullptr;
    State B{};
    Grave G{};
    uint8_t *dead = nullptr;
    KeyRec *krec = nullptr;
    OrdRec *orec = nullptr;
    uint32_t *hist = nullptr, *off = nullptr, *bsum = nullptr;
    double *H = nullptr, *GS = nullptr, *chunkS = nullptr, *chunkC = nullptr, *T = nullptr,
           *CR = nullptr, *tables = nullptr, *Eout = nullptr, *qpre = nullptr;
    int *chl = nullptr;
    double *chn = nullptr, *chg = nullptr;
    float *tables32 = nullptr;
    uint32_t *Eid = nullptr;
    Seg *seg = nullptr;
    Ctl *ctl = nullptr;
    uint32_t *tile_member = nullptr, *chunk_member = nullptr;
    Tables tb{};
    Map map{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool failed = false;
    size_t shared_bytes = 0;
    // one device allocation holds every array, the members' data pool last
    sim_allocator alloc{};      // caller's callbacks, or all NULL (hipMalloc / hipFree)
    void *arena = nullptr;
    size_t arena_bytes = 0;
    char *mdata = nullptr;      // members' drive, response and ion-profile arrays
    std::vector<Member> members;
    Ranges groups, chunks, buckets, mdata_units;   // mdata_units: 256-byte units of mdata
};

namespace {

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            return fail(SIM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                             \
    } while (0)

// Layout of the table block: 9 per-l arrays (ftil, wl, drive_w, self_w, nfA,
// nfB, lval, tl1, qmm, in this order), the two (l, m) triangles a_lm, b_lm
// (host side: N_lm and gamma_lm come from them), then at 32-byte aligned
// offsets the near-field constants (nf4, lg4) and the rescaled recurrence
// (fq4) with its zero entry.
constexpr int kQmmArray = 8;   // index of qmm among the per-l arrays

size_t nf4_offset(int L)
{
    const size_t base = (size_t)9 * (L + 1) + 2 * (size_t)((L + 1) * (L + 2) / 2);
    return (base + 3) & ~size_t(3);
}

size_t lg4_offset(int L) { return nf4_offset(L) + 4 * (size_t)(L + 1); }   // 32-byte aligned

size_t fq4_offset(int L) { return lg4_offset(L) + 4 * (size_t)(L + 1); }

// one zero entry after the fq4 triangle: the moments kernel reads one ahead
size_t tables_len(int L) { return fq4_offset(L) + 4 * (size_t)((L + 1) * (L + 2) / 2 + 1); }

// FP32 copies of the field kernel's tables, each at a 16-byte aligned offset:
// the axisymmetric near-field constants, the full near-field Legendre
// constants, the far-field recurrence.
size_t nf4_32_offset(int) { return 0; }

size_t lg4_32_offset(int L) { return nf4_32_offset(L) + 4 * (size_t)(L + 1); }

size_t fq4_32_offset(int L) { return lg4_32_offset(L) + 4 * (size_t)(L + 1); }

size_t lw4_32_offset(int L) { return fq4_32_offset(L) + 4 * (size_t)((L + 1) * (L + 2) / 2); }

size_t tables32_len(int L) { return lw4_32_offset(L) + 4 * (size_t)(L + 1); }

void plan_alloc(sim *h, Alloc &al, size_t pool_bytes)
{
    const Layout &lo = h->lo;
    const size_t n = (size_t)lo.n_tiles * kWave;
    al.add(&h->A, n);
    al.add(&h->B.x, n); al.add(&h->B.y, n); al.add(&h->B.z, n);
    al.add(&h->B.vx, n); al.add(&h->B.vy, n); al.add(&h->B.vz, n);
    al.add(&h->B.uid, n);
    al.add(&h->G.x, n); al.add(&h->G.y, n); al.add(&h->G.z, n);
    al.add(&h->G.vx, n); al.add(&h->G.vy, n); al.add(&h->G.vz, n);
    al.add(&h->G.uid, n);
    al.add(&h->dead, n);
    al.add(&h->krec, n);
    al.add(&h->orec, n);
    al.add(&h->hist, (size_t)lo.nb + 1);
    al.add(&h->off, (size_t)lo.nb + 1);
    al.add(&h->bsum, (size_t)lo.nb_blocks + 1);
    al.add(&h->H, (size_t)lo.n_tiles * (4 * lo.C + 2));
    al.add(&h->GS, (size_t)lo.n_groups * (lo.C2 + 1));
    al.add(&h->CR, (size_t)lo.n_groups * std::max(lo.C2, 1));
    al.add(&h->qpre, (size_t)lo.n_groups);
    al.add(&h->tables32, tables32_len(lo.L));
    al.add(&h->chunkS, (size_t)lo.n_chunks * (lo.C2 + 1));
    al.add(&h->chunkC, (size_t)lo.n_chunks * (lo.C2 + 1));
    al.add(&h->T, (size_t)lo.n_members * std::max(lo.C, 1));
    al.add(&h->tables, tables_len(lo.L));
    al.add(&h->chl, (size_t)std::max(lo.C, 1));
    al.add(&h->chn, (size_t)std::max(lo.C, 1));
    al.add(&h->chg, (size_t)std::max(lo.C, 1));
    al.add(&h->Eout, 3 * n);
    al.add(&h->Eid, n);
    al.add(&h->seg, (size_t)lo.n_members);
    al.add(&h->ctl, (size_t)lo.n_members);
    al.add(&h->tile_member, (size_t)lo.n_tiles);
    al.add(&h->chunk_member, (size_t)lo.n_chunks);
    al.add(&h->mdata, std::max<size_t>(pool_bytes, kPoolUnit));
}

// Host-side coefficient tables.  f_l and b^P_l are the closed forms of App. A
// and Sec. 3 (R = 1, R_E = a); c_l, the Legendre coefficients of the
// electrode data 1/2 sgn(cos th), are taken as (P_{l-1}(0) - P_{l+1}(0))/2.
std::vector<double> build_tables(const sim_params &p, const Layout &lo)
{
    const int L = lo.L;
    const double a = 1.0 - p.d, eps = p.eps_r;
    std::vector<double> t(tables_len(L), 0.0);
    double *ftil = t.data(), *wl = ftil + (L + 1), *drive = wl + (L + 1), *selfw = drive + (L + 1),
           *nfA = selfw + (L + 1), *nfB = nfA + (L + 1), *lval = nfB + (L + 1), *tl1 = lval + (L + 1),
           *qmm = tl1 + (L + 1), *alm = qmm + (L + 1),
           *blm = alm + (L + 1) * (L + 2) / 2, *nf4 = t.data() + nf4_offset(L);
    // Legendre values at 0 up to L + 1
    std::vector<double> p0(L + 3, 0.0);
    p0[0] = 1.0;
    if (L + 2 >= 1) p0[1] = 0.0;
    for (int l = 1; l + 1 <= L + 2; ++l) p0[l + 1] = -(double)l / (l + 1.0) * p0[l - 1];
    for (int l = 0; l <= L; ++l) {
        const double a2l1 = std::pow(a, 2.0 * l + 1.0);
        const double f = (l * (eps - 1.0) + (l + eps + l * eps) * a2l1) /
                         ((l + 1.0 + l * eps) + (l + 1.0) * (eps - 1.0) * a2l1);
        const double bP = (2.0 * l + 1.0) * eps * std::pow(a, l + 1.0) /
                          ((l + 1.0) * (eps - 1.0) * a2l1 + l * eps + l + 1.0);
        const double c = (l % 2 == 1) ? 0.5 * (p0[l - 1] - p0[l + 1]) : 0.0;
        ftil[l] = (l == 0) ? 0.0 : f;
        wl[l] = 1.0 / (2.0 * l + 1.0);
        drive[l] = c * bP * std::sqrt(4.0 * kPi / (2.0 * l + 1.0));
        selfw[l] = (l == 0) ? 0.0 : f / (4.0 * kPi);
        nfA[l] = (2.0 * l + 1.0) / (l + 1.0);
        nfB[l] = (double)l / (l + 1.0);
        lval[l] = (double)l;
        tl1[l] = 2.0 * l + 1.0;
        nf4[4 * l + 0] = nfA[l];
        nf4[4 * l + 1] = nfB[l];
        nf4[4 * l + 2] = tl1[l];
        nf4[4 * l + 3] = lval[l];
    }
    // Q_m^m = sqrt((2m+1)/(4 pi) / (2m)!) (2m-1)!! (sqrt 2 for m > 0)
    qmm[0] = 1.0 / std::sqrt(4.0 * kPi);
    for (int m = 1; m <= L; ++m) {
        double v = qmm[m - 1] * std::sqrt((2.0 * m + 1.0) / (2.0 * m));
        if (m == 1) v *= std::sqrt(2.0);
        qmm[m] = v;
    }
    for (int m = 0; m <= L; ++m) {
        for (int l = m + 1; l <= L; ++l) {
            const double l2 = (double)l * l, m2 = (double)m * m;
            alm[tri(l, m)] = std::sqrt((4.0 * l2 - 1.0) / (l2 - m2));
            blm[tri(l, m)] = (l >= m + 2)
                ? std::sqrt(((l - 1.0) * (l - 1.0) - m2) * (2.0 * l + 1.0) / ((l2 - m2) * (2.0 * l - 3.0)))
                : 0.0;
        }
    }
    // P_l = c_l Ph_l with c_0 = 1, c_l = c_{l-1} (2l-1)/l: the three-term
    // recurrence l P_l = (2l-1) u P_{l-1} - (l-1) P_{l-2} becomes
    // Ph_l = u Ph_{l-1} - gamma_l Ph_{l-2}, gamma_l = (l-1)^2 / ((2l-1)(2l-3));
    // P'_{l+1} = P'_{l-1} + (2l+1) c_l Ph_l
    double *lg = t.data() + lg4_offset(L);
    for (int l = 0; l <= L; ++l) {
        double c = 1.0;
        for (int k = 1; k <= l; ++k) c *= (2.0 * k - 1.0) / k;
        lg[4 * l + 0] = c;
        lg[4 * l + 1] = l * c;
        lg[4 * l + 2] = (double)l * l / ((2.0 * l + 1.0) * (2.0 * l - 1.0));
        lg[4 * l + 3] = (2.0 * l + 1.0) * c;
    }
    // rescaled far-field recurrence: Q_l^m = N_lm Qh_l^m with N_mm = Q_m^m and
    // N_lm = a_lm N_{l-1,m}, so gamma_lm = b_lm / (a_lm a_{l-1,m})
    double *fq = t.data() + fq4_offset(L);
    for (int m = 0, j = 0; m <= L; ++m) {
        for (int l = m; l <= L; ++l, ++j) {
            fq[4 * j] = (l >= m + 2) ? blm[tri(l, m)] / (alm[tri(l, m)] * alm[tri(l - 1, m)]) : 0.0;
            fq[4 * j + 1] = (double)(l - m);
            fq[4 * j + 2] = (double)(l + m + 1);
            fq[4 * j + 3] = 0.0;
        }
    }
    return t;
}

int launch_step(sim *h, hipStream_t s, bool field_only, hipEvent_t *ev)
{
    const Layout &lo = h->lo;
    const Extent &ex = h->ext;
    KParams kp = h->kp;
    kp.field_only = field_only ? 1 : 0;
    kp.fuse_keys = lo.tu.keys != 0 ? (lo.tu.keys > 0 ? 1 : 0)
                                   : (ex.n_tiles >= kFuseKeysMinTiles ? 1 : 0);
    kp.n_tiles = ex.n_tiles;
    kp.n_groups = ex.n_tiles / kTilesPerGroup;
    kp.n_chunks = ex.n_chunks;
    kp.nb = ex.nb;
    kp.n_members = ex.n_members;
    const Map &mp = h->map;
    const unsigned n = (unsigned)ex.n_tiles * kWave;
    const unsigned gN = (n + kBlock - 1) / kBlock;
    const unsigned gT = (unsigned)(ex.n_tiles / kTilesPerGroup);   // one block per group
    const unsigned gC = (unsigned)((lo.C2 + 1 + kBlock - 1) / kBlock);   // group-sum columns
    const unsigned gM = (unsigned)((ex.n_members + kBlock - 1) / kBlock);
    int e = 0;
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], s);
    };
    mark(KN_SORT_KEY);
    k_sort_key<<<gN, kBlock, 0, s>>>(mp, h->A, h->dead, h->krec, h->hist, kp);
    if (ex.nb_blocks <= kScanSingleMaxBlocks) {
        mark(KN_SCAN_A);
        mark(KN_SCAN_C);
        k_scan_single<<<1, kBlock, 0, s>>>(h->hist, h->off, ex.nb);
    } else {
        mark(KN_SCAN_A);
        k_scan_a<<<ex.nb_blocks, kBlock, 0, s>>>(h->hist, h->bsum, ex.nb);
        mark(KN_SCAN_C);
        k_scan_c<<<ex.nb_blocks, kBlock, 0, s>>>(h->hist, h->bsum, h->off, ex.nb);
    }
    mark(KN_SORT_SCATTER);
    k_sort_scatter<<<gN, kBlock, 0, s>>>(mp, h->krec, h->off, h->orec, kp);
    mark(KN_SORT_RANK);
    k_sort_rank_move<<<gN, kBlock, 0, s>>>(mp, h->orec, h->off, h->A, h->B, kp);
    mark(KN_MOMENTS);
    if (lo.full) k_moments<true><<<gT, kBlock, 0, s>>>(mp, h->B, h->tb, kp, h->H, h->GS);
    else k_moments<false><<<gT, kBlock, 0, s>>>(mp, h->B, h->tb, kp, h->H, h->GS);
    mark(KN_CHUNK_SUMS);
    k_chunk_sums<<<dim3(ex.n_chunks, gC), kBlock, 0, s>>>(mp, h->GS, h->chunkS, kp);
    mark(KN_CHUNK_SCAN);
    k_chunk_scan<<<dim3((lo.C2 + 1 + kWavesPerBlock - 1) / kWavesPerBlock, ex.n_members), kBlock, 0,
                   s>>>(mp, h->chunkS, h->chunkC, h->T, kp);
    mark(KN_CHUNK_APPLY);
    k_chunk_apply<<<dim3(ex.n_chunks, gC), kBlock, 0, s>>>(mp, h->GS, h->chunkC, h->T, h->tb, kp,
                                                           h->CR, h->qpre);
    mark(KN_FIELD_PUSH);
#define MRP_FIELD(FULLV, FO, F32, N64)                                                   \
    k_field_push<FULLV, FO, F32, N64><<<gT, kBlock, 0, s>>>(mp, h->B, h->A, h->dead, h->G, \
                                                            h->H, h->CR, h->qpre,          \
                                                            h->tb, kp, h->Eout, h->Eid,    \
                                                            h->krec, h->hist)
#define MRP_FIELD_P(FULLV, FO)                                           \
    do {                                                                 \
        if (lo.near64) MRP_FIELD(FULLV, FO, true, true);                 \
        else if (lo.fp32) MRP_FIELD(FULLV, FO, true, false);             \
        else MRP_FIELD(FULLV, FO, false, false);                         \
    } while (0)
    if (field_only) {
        if (lo.full) MRP_FIELD_P(true, true);
        else MRP_FIELD_P(false, true);
    } else {
        if (lo.full) MRP_FIELD_P(true, false);
        else MRP_FIELD_P(false, false);
        mark(KN_STEP_FINISH);
        k_step_finish<<<gM, kBlock, 0, s>>>(mp, kp);
    }
    if (ev) (void)hipEventRecord(ev[KN_COUNT], s);
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) e = fail(SIM_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
    return e;
}

// Give a member's range of the data pool back (no device call).
void free_member_arrays(sim *h, Member &m)
{
    if (m.md_units) h->mdata_units.give(m.md_start, m.md_units);
    m.md_units = 0;
    m.seg.u_asy = nullptr;
    m.seg.qdiff = nullptr;
    m.seg.ion_tab = nullptr;
}

// The handle's work completes before its graph and memory go: the stream is
// drained first.
void release(sim *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->exec = nullptr;
    h->graph = nullptr;
    if (h->arena) {
        void *as = h->own_stream ? nullptr : (void *)h->stream;   // the stream given to alloc
        if (h->alloc.free) h->alloc.free(h->alloc.ctx, h->arena, h->arena_bytes, as);
        else (void)hipFree(h->arena);
    }
    h->arena = nullptr;
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    h->cap_stream = nullptr;
    h->stream = nullptr;
}

int check_handle(sim *h)
{
    if (!h) return fail(SIM_ESTATE, "NULL handle");
    if (h->failed) return fail(SIM_ESTATE, "handle is in the failed state");
    return SIM_OK;
}

int mark_failed(sim *h, int code)
{
    if (code == SIM_EDEVICE) h->failed = true;
    return code;
}

int check_member_index(sim *h, int32_t index)
{
    if (index < 0 || index >= (int32_t)h->members.size() || !h->members[index].used)
        return fail(SIM_ERANGE, "no member at index " + std::to_string(index));
    return SIM_OK;
}

// The host-side constant tables of a layout: the FP64 block of
// build_tables, its FP32 copies, and the degree and normalisation of each
// channel in stream order.
struct HostTables {
    std::vector<double> tab;
    std::vector<float> tab32;
    std::vector<int> chl;
    std::vector<double> chn, chg;
};

int make_host_tables(const sim_params &p, const Layout &lo, HostTables *ht)
{
    const int L = lo.L;
    ht->tab = build_tables(p, lo);
    const std::vector<double> &tab = ht->tab;
    std::vector<float> &tab32 = ht->tab32;
    tab32.assign(tables32_len(L), 0.f);
    {
        const size_t ntri = (size_t)(L + 1) * (L + 2) / 2;
        const double *nf4 = tab.data() + nf4_offset(L);
        for (int i = 0; i < 4 * (L + 1); ++i) tab32[nf4_32_offset(L) + i] = (float)nf4[i];
        const double *lg = tab.data() + lg4_offset(L);
        for (int i = 0; i < 4 * (L + 1); ++i) tab32[lg4_32_offset(L) + i] = (float)lg[i];
        const double *fq = tab.data() + fq4_offset(L);
        for (size_t i = 0; i < 4 * ntri; ++i) tab32[fq4_32_offset(L) + i] = (float)fq[i];
        float *lw = tab32.data() + lw4_32_offset(L);
        for (int l = 0; l <= L; ++l) {
            lw[4 * l + 0] = (float)(1.0 / (l + 1.0));
            lw[4 * l + 1] = 0.0f;
            lw[4 * l + 2] = (float)(2.0 * l + 1.0);
            lw[4 * l + 3] = (float)(l + 1.0);
        }
    }
    // degree of each channel in stream order (m outer, l = max(m,1)..L inner)
    // and its far-field normalisation N_lm
    std::vector<int> &chl = ht->chl;
    std::vector<double> &chn = ht->chn;
    chl.clear();
    chn.clear();
    {
        const double *qmm = tab.data() + kQmmArray * (L + 1);
        const double *alm = qmm + (L + 1);
        for (int m = 0; m <= (lo.full ? L : 0); ++m) {
            double nlm = qmm[m];   // N_mm
            for (int l = m; l <= L; ++l) {
                if (l > m) nlm *= alm[tri(l, m)];
                if (l == 0) continue;
                for (int sc = 0; sc < (m > 0 ? 2 : 1); ++sc) {
                    chl.push_back(l);
                    chn.push_back(nlm);
                }
            }
        }
    }
    if ((int)chl.size() != lo.C) return fail(SIM_EDEVICE, "channel count mismatch");
    // N_lm^2 / (2l+1): a raw sum of Qh to a field coefficient (times 1 / ntilde)
    ht->chg.resize(chl.size());
    for (size_t c = 0; c < chl.size(); ++c) ht->chg[c] = chn[c] * chn[c] / (2.0 * chl[c] + 1.0);
    if (chl.empty()) {
        chl.push_back(0);
        chn.push_back(0.0);
        ht->chg.push_back(0.0);
    }
    return SIM_OK;
}

// Point the kernels' table, parameter and map views at the handle's carved
// arrays (its layout set).
void bind_device_tables(sim *h)
{
    const Layout &lo = h->lo;
    const int L = lo.L;
    double *tb = h->tables;
    h->tb.ftil = tb;
    h->tb.wl = tb + (L + 1);
    h->tb.drive_w = tb + 2 * (L + 1);
    h->tb.self_w = tb + 3 * (L + 1);
    h->tb.nfA = tb + 4 * (L + 1);
    h->tb.nfB = tb + 5 * (L + 1);
    h->tb.nf4 = reinterpret_cast<const double4 *>(tb + nf4_offset(L));
    h->tb.lg4 = reinterpret_cast<const double4 *>(tb + lg4_offset(L));
    h->tb.fq4 = reinterpret_cast<const double4 *>(tb + fq4_offset(L));
    h->tb.chn = h->chn;
    h->tb.chl = h->chl;
    h->tb.chg = h->chg;
    h->tb.nf4_32 = reinterpret_cast<const float4 *>(h->tables32 + nf4_32_offset(L));
    h->tb.lg4_32 = reinterpret_cast<const float4 *>(h->tables32 + lg4_32_offset(L));
    h->tb.fq4_32 = reinterpret_cast<const float4 *>(h->tables32 + fq4_32_offset(L));
    h->tb.lw4_32 = reinterpret_cast<const float4 *>(h->tables32 + lw4_32_offset(L));
    KParams &kp = h->kp;
    kp.L = lo.L;
    kp.C = lo.C;
    kp.C2 = lo.C2;
    kp.SW = lo.C2 + 1;
    kp.HW = 4 * lo.C + 2;
    kp.n_tiles = lo.n_tiles;
    kp.n_groups = lo.n_groups;
    kp.n_chunks = lo.n_chunks;
    kp.nb = lo.nb;
    kp.n_members = lo.n_members;
    kp.fp32 = lo.fp32 ? 1 : 0;
    kp.field_only = 0;
    kp.fuse_keys = 0;
    h->map.seg = h->seg;
    h->map.ctl = h->ctl;
    h->map.tile_member = h->tile_member;
    h->map.chunk_member = h->chunk_member;
}

// Carve the arrays of plan_alloc out of one block at base, in order, each
// 256-byte aligned.
void carve(Alloc &al, void *base)
{
    char *at = static_cast<char *>(base);
    for (auto &it : al.items) {
        *it.first = at;
        at += align_unit(it.second);
    }
}

// Allocate the arena (the shared arrays and the members' data pool, in one
// allocation from the caller's allocator or hipMalloc), upload the tables.
int engine_init(sim *h, const sim_params *p, const Layout &lo, void *hip_stream,
                const sim_allocator *alloc, size_t pool_bytes)
{
    h->prm = *p;
    h->lo = lo;
    if (alloc) {
        if (!alloc->alloc || !alloc->free)
            return fail(SIM_EINVAL, "sim_allocator needs both alloc and free");
        h->alloc = *alloc;
    }
    Alloc al;
    plan_alloc(h, al, pool_bytes);
    h->shared_bytes = al.total();
    if (p->mem_limit_bytes && h->shared_bytes > p->mem_limit_bytes)
        return fail(SIM_ENOMEM, "footprint " + std::to_string(h->shared_bytes) +
                                    " B exceeds mem_limit_bytes");
    // the arena first (before any stream exists: a caller's allocator that
    // fails leaves no device state behind); its stream is the caller's, or
    // NULL when the handle runs on a stream of its own
    h->arena_bytes = h->shared_bytes;
    if (h->alloc.alloc) {
        h->arena = h->alloc.alloc(h->alloc.ctx, h->arena_bytes, hip_stream);
        if (!h->arena) return fail(SIM_ENOMEM, "the caller's allocator returned NULL");
        if (reinterpret_cast<uintptr_t>(h->arena) % kPoolUnit) {
            h->alloc.free(h->alloc.ctx, h->arena, h->arena_bytes, hip_stream);
            h->arena = nullptr;
            return fail(SIM_EINVAL, "the caller's allocator must return 256-byte aligned memory");
        }
    } else {
        hipError_t e = hipMalloc(&h->arena, h->arena_bytes);
        if (e != hipSuccess) {
            h->arena = nullptr;
            return fail(SIM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    carve(al, h->arena);
    h->mdata_units.reset((uint32_t)(std::max<size_t>(pool_bytes, kPoolUnit) / kPoolUnit));
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
            return fail(SIM_EDEVICE, "hipStreamCreate failed");
        h->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(SIM_EDEVICE, "hipStreamCreate failed");

    HostTables ht;
    if (int rc = make_host_tables(*p, lo, &ht)) return rc;
    bind_device_tables(h);
    h->groups.reset((uint32_t)lo.n_groups);
    h->chunks.reset((uint32_t)lo.n_chunks);
    h->buckets.reset((uint32_t)lo.nb);
    h->members.assign((size_t)lo.n_members, Member());

    std::vector<Seg> segs((size_t)lo.n_members);   // used = 0
    std::vector<Ctl> ctls((size_t)lo.n_members);
    std::vector<uint32_t> none_t((size_t)lo.n_tiles, kNone), none_c((size_t)lo.n_chunks, kNone);
    if (hipMemcpy(h->tables, ht.tab.data(), sizeof(double) * ht.tab.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->chl, ht.chl.data(), sizeof(int) * ht.chl.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->chn, ht.chn.data(), sizeof(double) * ht.chn.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->chg, ht.chg.data(), sizeof(double) * ht.chg.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->tables32, ht.tab32.data(), sizeof(float) * ht.tab32.size(),
                  hipMemcpyHostToDevice) ||
        hipMemcpy(h->seg, segs.data(), sizeof(Seg) * segs.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->ctl, ctls.data(), sizeof(Ctl) * ctls.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->tile_member, none_t.data(), 4 * none_t.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->chunk_member, none_c.data(), 4 * none_c.size(), hipMemcpyHostToDevice) ||
        hipMemset(h->dead, 0, (size_t)lo.n_tiles * kWave) ||
        hipMemset(h->hist, 0, sizeof(uint32_t) * ((size_t)lo.nb + 1)))
        return fail(SIM_EDEVICE, "upload failed");

    if (hipDeviceSynchronize() != hipSuccess) return fail(SIM_EDEVICE, "device sync failed");
    return SIM_OK;
}

// Recompute the extent in use and, when it changed (or no graph exists yet),
// capture one step into a new graph.  The handle's stream is idle here.
int update_graph(sim *h)
{
    Extent ex;
    for (int32_t k = 0; k < (int32_t)h->members.size(); ++k) {
        const Member &m = h->members[k];
        if (!m.used) continue;
        ex.n_tiles = std::max(ex.n_tiles, (int)(m.seg.t0 + m.seg.nt));
        ex.n_chunks = std::max(ex.n_chunks, (int)(m.seg.c0 + m.seg.nc));
        ex.nb = std::max(ex.nb, (int)(m.seg.b0 + m.seg.nb));
        ex.n_members = std::max(ex.n_members, k + 1);
    }
    ex.nb_blocks = (ex.nb + kScanPerBlock - 1) / kScanPerBlock;
    if (h->exec && ex == h->ext) return SIM_OK;
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->exec = nullptr;
    h->graph = nullptr;
    h->ext = ex;
    if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return mark_failed(h, fail(SIM_EDEVICE, "hipStreamBeginCapture failed"));
    int le = launch_step(h, h->cap_stream, false, nullptr);
    hipError_t ce = hipStreamEndCapture(h->cap_stream, &h->graph);
    if (le != SIM_OK) return mark_failed(h, le);
    if (ce != hipSuccess)
        return mark_failed(h, fail(SIM_EDEVICE, std::string("capture: ") + hipGetErrorString(ce)));
    if (hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) != hipSuccess)
        return mark_failed(h, fail(SIM_EDEVICE, "hipGraphInstantiate failed"));
    return SIM_OK;
}

// A member's host-side data after validation: ids and the id -> creation
// index map.
struct Prepared {
    std::vector<uint32_t> uid;
    std::vector<std::pair<uint32_t, int64_t>> idx;
};

// Validate a member completely (no device work).
int prepare_member(const sim_member *m, Prepared *pr)
{
    std::string why;
    if (!check_member_scalars(m, &why)) return fail(SIM_EINVAL, why);
    const int64_t n = m->n;
    if (!m->pos || !m->vel) return fail(SIM_EINVAL, "pos and vel are required");
    if (m->n_steps > 0 && !m->u_asy) return fail(SIM_EINVAL, "u_asy is required when n_steps > 0");
    for (int64_t i = 0; i < n; ++i) {
        const double *x = m->pos + 3 * i, *v = m->vel + 3 * i;
        for (int j = 0; j < 3; ++j)
            if (!std::isfinite(x[j]) || !std::isfinite(v[j]))
                return fail(SIM_EINVAL, "non-finite particle state at index " + std::to_string(i));
        const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (!(r > 1.0 && r < m->r_out))
            return fail(SIM_EINVAL, "particle " + std::to_string(i) + " not inside 1 < r < r_out");
    }
    for (int64_t s = 0; s < m->n_steps; ++s)
        if (!std::isfinite(m->u_asy[s])) return fail(SIM_EINVAL, "non-finite u_asy");
    if (m->ion_profile)
        for (int64_t j = 0; j < m->ion_profile_len; ++j)
            if (!std::isfinite(m->ion_profile[j]) || m->ion_profile[j] < 0.0)
                return fail(SIM_EINVAL, "ion_profile values must be finite and >= 0");
    pr->uid.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) pr->uid[i] = m->ids ? m->ids[i] : (uint32_t)i;
    if (!(m->ion_mass > 0.0))
        for (int64_t i = 0; i < n; ++i)
            if (pr->uid[i] & kIonBit) return fail(SIM_EINVAL, "ion ids (bit 31) need ion_mass > 0");
    pr->idx.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) pr->idx[i] = {pr->uid[i], i};
    std::sort(pr->idx.begin(), pr->idx.end());
    for (int64_t i = 1; i < n; ++i)
        if (pr->idx[i].first == pr->idx[i - 1].first) return fail(SIM_EINVAL, "ids are not distinct");
    return SIM_OK;
}

// Place and upload one validated member.  On failure the handle is unchanged
// (apart from the device contents of free ranges).
int engine_add(sim *h, const sim_member *m, Prepared &pr, int32_t *index)
{
    const int64_t n = m->n;
    std::vector<uint32_t> &uid = pr.uid;
    int32_t slot = -1;
    for (int32_t k = 0; k < (int32_t)h->members.size(); ++k)
        if (!h->members[k].used) { slot = k; break; }
    if (slot < 0) return fail(SIM_ENOMEM, "member table is full");
    const size_t mbytes = member_bytes(m->n_steps, m->ion_profile ? m->ion_profile_len : 0);
    const uint32_t md_units = (uint32_t)(mbytes / kPoolUnit);
    const MemberShape sh = member_shape(n, h->lo.tu);
    uint32_t g0 = 0, c0 = 0, b0 = 0, md0 = 0;
    if (!h->groups.take(sh.ng, &g0)) return fail(SIM_ENOMEM, "no free slot range for the member");
    if (!h->chunks.take(sh.nc, &c0)) {
        h->groups.give(g0, sh.ng);
        return fail(SIM_ENOMEM, "no free chunk range for the member");
    }
    if (!h->buckets.take(sh.nb, &b0)) {
        h->groups.give(g0, sh.ng);
        h->chunks.give(c0, sh.nc);
        return fail(SIM_ENOMEM, "no free bucket range for the member");
    }
    if (!h->mdata_units.take(md_units, &md0)) {
        h->groups.give(g0, sh.ng);
        h->chunks.give(c0, sh.nc);
        h->buckets.give(b0, sh.nb);
        return fail(SIM_ENOMEM, "the batch's member data pool has no room for the member's "
                                "drive and response arrays");
    }
    Member mb;
    mb.md_start = md0;
    mb.md_units = md_units;
    mb.used = true;
    mb.n = n;
    mb.step_host = m->start_step;
    mb.start_step = m->start_step;
    mb.q_surface0 = m->q_surface0;
    mb.id_index = std::move(pr.idx);
    Seg &sg = mb.seg;
    const uint32_t t0 = g0 * kTilesPerGroup;
    sg.p0 = g0 * kGroupSlots;
    sg.cap = sh.ng * kGroupSlots;
    sg.t0 = t0;
    sg.nt = sh.nt;
    sg.g0 = g0;
    sg.ng = sh.ng;
    sg.c0 = c0;
    sg.nc = sh.nc;
    sg.cl = sh.cl;
    sg.b0 = b0;
    sg.nb = sh.nb;
    sg.inv_vol = 1.0 / (m->r_out * m->r_out * m->r_out - 1.0);
    sg.ntilde = m->ntilde;
    sg.inv_ntilde = 1.0 / m->ntilde;
    sg.ion_density = m->ion_density;
    sg.q_surface0 = m->q_surface0;
    sg.dt = m->dt;
    sg.r_out = m->r_out;
    sg.seed = m->seed;
    sg.probe_bc = m->probe_bc;
    sg.wall_bc = m->wall_bc;
    sg.n_steps = m->n_steps;
    sg.ion_qm = m->ion_mass > 0.0 ? 1.0 / m->ion_mass : 0.0;
    sg.near_w = near_width(h->lo.tu, h->lo.fp32, h->lo.L, n);
    sg.used = 1;
    auto undo = [&](int code) {
        free_member_arrays(h, mb);
        h->groups.give(g0, sh.ng);
        h->chunks.give(c0, sh.nc);
        h->buckets.give(b0, sh.nb);
        return code;
    };
    const size_t ns = (size_t)std::max<int64_t>(m->n_steps, 1);
    char *md = h->mdata + (size_t)md0 * kPoolUnit;
    double *u_dev = reinterpret_cast<double *>(md);
    double *q_dev = reinterpret_cast<double *>(md + align_unit(8 * ns));
    sg.u_asy = u_dev;
    sg.qdiff = q_dev;
    std::vector<double> ion_tab;
    if (m->ion_profile) {
        // node densities, then the enclosed charge at every node, segment by
        // segment in closed form (the same expression as the field kernel at
        // dd = h)
        const int64_t K = m->ion_profile_len - 1;
        const double h = (m->r_out - 1.0) / (double)K;
        ion_tab.assign(2 * (size_t)(K + 1), 0.0);
        for (int64_t j = 0; j <= K; ++j) ion_tab[j] = m->ion_profile[j];
        double q = 0.0;
        for (int64_t j = 0; j < K; ++j) {
            ion_tab[K + 1 + j] = q;
            const double rj = 1.0 + (double)j * h, dd = h, d2 = dd * dd;
            const double nj = m->ion_profile[j], beta = (m->ion_profile[j + 1] - nj) / h;
            const double seg = nj * (rj * rj * dd + rj * d2 + d2 * dd / 3.0) +
                               beta * (rj * rj * d2 / 2.0 + 2.0 * rj * d2 * dd / 3.0 + d2 * d2 / 4.0);
            q += 4.0 * kPi * m->ntilde * seg;
        }
        ion_tab[2 * K + 1] = q;
        sg.ion_tab = reinterpret_cast<double *>(md + 2 * align_unit(8 * ns));
        sg.ion_k = (int32_t)K;
        sg.ion_h = h;
        sg.ion_inv_h = (double)K / (m->r_out - 1.0);
    }

    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        h->failed = true;
        return undo(fail(SIM_EDEVICE, "stream synchronisation failed"));
    }
    std::vector<PRec> recs((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        PRec &r = recs[i];
        r.x = m->pos[3 * i];
        r.y = m->pos[3 * i + 1];
        r.z = m->pos[3 * i + 2];
        r.vx = m->vel[3 * i];
        r.vy = m->vel[3 * i + 1];
        r.vz = m->vel[3 * i + 2];
        r.uid = uid[i];
        r.pad[0] = r.pad[1] = r.pad[2] = 0u;
    }
    Ctl ctl{};
    ctl.step = m->start_step;
    ctl.n_cur = (uint32_t)n;
    ctl.n_live = (uint32_t)n;
    ctl.n_dead = 0;
    ctl.q_surface = m->q_surface0;
    std::vector<double> zeros(ns, 0.0);
    std::vector<uint32_t> tm(sh.nt, (uint32_t)slot), cm(sh.nc, (uint32_t)slot);
    if (hipMemcpy(h->A + sg.p0, recs.data(), sizeof(PRec) * n, hipMemcpyHostToDevice) ||
        hipMemset(h->dead + sg.p0, 0, sg.cap) ||
        hipMemcpy(q_dev, zeros.data(), 8 * ns, hipMemcpyHostToDevice) ||
        (m->n_steps > 0 && hipMemcpy(u_dev, m->u_asy, 8 * m->n_steps, hipMemcpyHostToDevice)) ||
        (!ion_tab.empty() && hipMemcpy((void *)sg.ion_tab, ion_tab.data(), 8 * ion_tab.size(),
                                       hipMemcpyHostToDevice)) ||
        hipMemcpy(h->ctl + slot, &ctl, sizeof(Ctl), hipMemcpyHostToDevice) ||
        hipMemcpy(h->tile_member + t0, tm.data(), 4 * tm.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->chunk_member + c0, cm.data(), 4 * cm.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->seg + slot, &sg, sizeof(Seg), hipMemcpyHostToDevice)) {
        h->failed = true;
        return undo(fail(SIM_EDEVICE, "member upload failed"));
    }
    h->members[slot] = std::move(mb);
    *index = slot;
    return SIM_OK;
}

int engine_remove(sim *h, int32_t index)
{
    int rc = check_member_index(h, index);
    if (rc) return rc;
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        h->failed = true;
        return fail(SIM_EDEVICE, "stream synchronisation failed");
    }
    Member &mb = h->members[index];
    Seg off{};   // used = 0
    std::vector<uint32_t> tm(mb.seg.nt, kNone), cm(mb.seg.nc, kNone);
    // the member's last push may have counted its particles into its buckets
    // for a next step; the buckets go back to the pool cleared
    if (hipMemcpy(h->seg + index, &off, sizeof(Seg), hipMemcpyHostToDevice) ||
        hipMemset(h->hist + mb.seg.b0, 0, sizeof(uint32_t) * mb.seg.nb) ||
        hipMemcpy(h->tile_member + mb.seg.t0, tm.data(), 4 * tm.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->chunk_member + mb.seg.c0, cm.data(), 4 * cm.size(), hipMemcpyHostToDevice)) {
        h->failed = true;
        return fail(SIM_EDEVICE, "member table update failed");
    }
    free_member_arrays(h, mb);
    h->groups.give(mb.seg.g0, mb.seg.ng);
    h->chunks.give(mb.seg.c0, mb.seg.nc);
    h->buckets.give(mb.seg.b0, mb.seg.nb);
    mb = Member();
    return SIM_OK;
}

int enqueue_steps(sim *h, int64_t k)
{
    for (int64_t i = 0; i < k; ++i) {
        hipError_t e = hipGraphLaunch(h->exec, h->stream);
        if (e != hipSuccess) {
            h->failed = true;
            return fail(SIM_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        }
    }
    for (Member &m : h->members)
        if (m.used) m.step_host = std::min(m.step_host + k, m.seg.n_steps);
    return SIM_OK;
}

sim_member member_from_params(const sim_params *p, int64_t n, const double *pos, const double *vel,
                              const uint32_t *ids, const double *u_asy, int64_t n_steps,
                              int64_t start_step)
{
    sim_member m;
    std::memset(&m, 0, sizeof(m));
    m.struct_size = sizeof(sim_member);
    m.n = n;
    m.pos = pos;
    m.vel = vel;
    m.ids = ids;
    m.u_asy = u_asy;
    m.n_steps = n_steps;
    m.start_step = start_step;
    m.ntilde = p->ntilde;
    m.ion_density = p->ion_density;
    m.q_surface0 = p->q_surface0;
    m.r_out = p->r_out;
    m.dt = p->dt;
    m.seed = p->seed;
    m.probe_bc = p->probe_bc;
    m.wall_bc = p->wall_bc;
    return m;
}

int64_t slots_for(int64_t n) { return (int64_t)groups_for(n) * kGroupSlots; }

// ---------------------------------------------------------------------------
// Field evaluation without allocation: every working array in a static
// device buffer
// ---------------------------------------------------------------------------

// One buffer per GPU the library runs on, held until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// Device address of this device's scratch (looked up once per device; the
// array's name in host code is a host-side stand-in, not this address).
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SIM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SIM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SIM_OK;
}

// The tables and control words a one-member handle would hold before its
// first step, written by a kernel (the buffer keeps the previous call's
// contents): the member's description, its control block, the tile and
// chunk maps, the absorbed flags and the bucket histogram cleared, and the
// drive value of the evaluated step.
__global__ void k_static_setup(Seg sg, Ctl ct, Seg *seg, Ctl *ctl, uint32_t *tile_member,
                               uint32_t *chunk_member, uint8_t *dead, uint32_t *hist,
                               double *u_dev, double u_asy, int n_tiles, int n_chunks, int nb)
{
    const int stride = gridDim.x * blockDim.x;
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = i0; i < n_tiles * kWave; i += stride) dead[i] = 0;
    for (int i = i0; i < n_tiles; i += stride) tile_member[i] = 0;
    for (int i = i0; i < n_chunks; i += stride) chunk_member[i] = 0;
    for (int i = i0; i <= nb; i += stride) hist[i] = 0;
    if (i0 == 0) {
        seg[0] = sg;
        ctl[0] = ct;
        u_dev[0] = u_asy;
    }
}

// Particle records from positions [3n] (particle-major), id = index.
__global__ void k_static_pack(const double *pos, uint32_t n, PRec *A)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    PRec r;
    r.x = pos[3 * (size_t)i];
    r.y = pos[3 * (size_t)i + 1];
    r.z = pos[3 * (size_t)i + 2];
    r.vx = r.vy = r.vz = 0.0;
    r.uid = i;
    r.pad[0] = r.pad[1] = r.pad[2] = 0u;
    A[i] = r;
}

// The field at sorted position p back to the particle's index (its id).
__global__ void k_static_unpack(const double *Eout, const uint32_t *Eid, uint32_t n, double *E)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const size_t k = Eid[p];
    E[3 * k] = Eout[3 * (size_t)p];
    E[3 * k + 1] = Eout[3 * (size_t)p + 1];
    E[3 * k + 2] = Eout[3 * (size_t)p + 2];
}

}  // namespace

extern "C" {

void sim_params_default(sim_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(sim_params);
    p->d = 0.25;
    p->eps_r = 4.0;
    p->r_out = 5.0;
    p->dt = 0.05;
    p->ntilde = 1.0;
    p->ion_density = 1.0;
    p->q_surface0 = 0.0;
    p->l_max = 8;
    p->m_mode = SIM_M_FULL;
    p->probe_bc = SIM_BC_ABSORB;
    p->wall_bc = SIM_BC_SPECULAR;
    p->precision = SIM_FP64;
    p->tile = 0;
    p->seed = 0;
    p->mem_limit_bytes = 0;
}

void sim_member_default(sim_member *m)
{
    if (!m) return;
    sim_params p;
    sim_params_default(&p);
    *m = member_from_params(&p, 0, nullptr, nullptr, nullptr, nullptr, 0, 0);
}

}  // extern "C"

namespace {

int64_t footprint(const sim_params *common, int64_t slots, int32_t max_members, int64_t chunks,
                  size_t pool_bytes)
{
    Layout lo;
    std::string why;
    if (!make_layout(common, slots, max_members, chunks, &lo, &why)) return fail(SIM_EINVAL, why);
    sim tmp;
    tmp.lo = lo;
    Alloc al;
    plan_alloc(&tmp, al, pool_bytes);
    return (int64_t)al.total();
}

}  // namespace

extern "C" {

int64_t sim_member_data_bytes(int64_t n_steps, int64_t ion_profile_len)
{
    if (n_steps < 0 || ion_profile_len < 0) return fail(SIM_EINVAL, "negative size");
    return (int64_t)member_bytes(n_steps, ion_profile_len);
}

int64_t sim_batch_footprint_bytes(const sim_params *common, int64_t slot_capacity,
                                  int32_t max_members, int64_t member_data_bytes)
{
    if (member_data_bytes < 0) return fail(SIM_EINVAL, "member_data_bytes < 0");
    return footprint(common, slot_capacity, max_members, -1, align_unit((size_t)member_data_bytes));
}

int64_t sim_footprint_bytes(const sim_params *p, int64_t n, int64_t n_steps)
{
    std::string why;
    if (!check_common(p, &why)) return fail(SIM_EINVAL, why);
    sim_member m = member_from_params(p, n, nullptr, nullptr, nullptr, nullptr, n_steps, 0);
    if (!check_member_scalars(&m, &why)) return fail(SIM_EINVAL, why);
    return footprint(p, slots_for(n), 1, member_shape(n, tuning_of(p)).nc,
                     member_bytes(n_steps, 0));
}

int sim_batch_create(const sim_params *common, int64_t slot_capacity, int32_t max_members,
                     int64_t member_data_bytes, int32_t n_members, const sim_member *members,
                     void *hip_stream, const sim_allocator *alloc, sim_t **out)
{
    if (!out) return fail(SIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_members < 0 || (n_members > 0 && !members)) return fail(SIM_EINVAL, "bad member list");
    if (member_data_bytes < 0) return fail(SIM_EINVAL, "member_data_bytes < 0");
    std::string why;
    if (!check_common(common, &why)) return fail(SIM_EINVAL, why);
    int64_t need = 0, chunks = 0;
    size_t pool_need = 0;
    std::vector<Prepared> prep((size_t)n_members);
    for (int32_t i = 0; i < n_members; ++i) {
        if (prepare_member(&members[i], &prep[i]))
            return fail(SIM_EINVAL, "member " + std::to_string(i) + ": " + g_last_error);
        need += slots_for(members[i].n);
        chunks += member_shape(members[i].n, tuning_of(common)).nc;
        pool_need += member_bytes(members[i].n_steps,
                                  members[i].ion_profile ? members[i].ion_profile_len : 0);
    }
    const size_t pool_bytes =
        member_data_bytes == 0 ? pool_need : align_unit((size_t)member_data_bytes);
    if (pool_bytes < pool_need)
        return fail(SIM_ENOMEM, "members need more member data bytes than member_data_bytes");
    // exactly the initial members, or room for any later mix
    const bool exact = slot_capacity == 0 && (max_members == 0 || max_members == n_members);
    if (max_members == 0) max_members = n_members;
    if (max_members < n_members) return fail(SIM_EINVAL, "max_members < n_members");
    if (slot_capacity == 0) slot_capacity = need;
    if (slot_capacity < need) return fail(SIM_ENOMEM, "members need more slots than slot_capacity");
    Layout lo;
    if (!make_layout(common, slot_capacity, max_members, exact ? chunks : -1, &lo, &why))
        return fail(SIM_EINVAL, why);
    sim *h = new (std::nothrow) sim();
    if (!h) return fail(SIM_ENOMEM, "host allocation failed");
    auto bail = [&](int code) {
        release(h);
        delete h;
        return code;
    };
    int rc = engine_init(h, common, lo, hip_stream, alloc, pool_bytes);
    if (rc) return bail(rc);
    for (int32_t i = 0; i < n_members; ++i) {
        int32_t idx = -1;
        rc = engine_add(h, &members[i], prep[i], &idx);
        if (rc) {
            const std::string msg = "member " + std::to_string(i) + ": " + g_last_error;
            bail(rc);
            return fail(rc, msg);
        }
    }
    rc = update_graph(h);
    if (rc) return bail(rc);
    *out = h;
    return SIM_OK;
}

int sim_create(const sim_params *p, int64_t n, const double *pos, const double *vel,
               const uint32_t *ids, const double *u_asy, int64_t n_steps, int64_t start_step,
               void *hip_stream, const sim_allocator *alloc, sim_t **out)
{
    if (!out) return fail(SIM_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!check_common(p, &why)) return fail(SIM_EINVAL, why);
    sim_member m = member_from_params(p, n, pos, vel, ids, u_asy, n_steps, start_step);
    if (!check_member_scalars(&m, &why)) return fail(SIM_EINVAL, why);
    if (p->mem_limit_bytes) {
        const int64_t fp = sim_footprint_bytes(p, n, n_steps);
        if (fp > (int64_t)p->mem_limit_bytes)
            return fail(SIM_ENOMEM, "footprint " + std::to_string(fp) + " B exceeds mem_limit_bytes");
    }
    return sim_batch_create(p, 0, 1, 0, 1, &m, hip_stream, alloc, out);
}

int sim_batch_add(sim_t *h, const sim_member *m, int32_t *index)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!index) return fail(SIM_EINVAL, "index is NULL");
    Prepared pr;
    rc = prepare_member(m, &pr);
    if (rc) return rc;
    rc = engine_add(h, m, pr, index);
    if (rc) return rc;
    return update_graph(h);
}

int sim_batch_remove(sim_t *h, int32_t index)
{
    int rc = check_handle(h);
    if (rc) return rc;
    rc = engine_remove(h, index);
    if (rc) return rc;
    return update_graph(h);
}

int sim_step(sim_t *h, int64_t k)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (k < 0) return fail(SIM_EINVAL, "k < 0");
    for (const Member &m : h->members)
        if (m.used && m.step_host + k > m.seg.n_steps) return fail(SIM_ERANGE, "steps beyond n_steps");
    return enqueue_steps(h, k);
}

int sim_batch_step(sim_t *h, int64_t k)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (k < 0) return fail(SIM_EINVAL, "k < 0");
    int64_t left = 0;
    for (const Member &m : h->members)
        if (m.used) left = std::max(left, m.seg.n_steps - m.step_host);
    return enqueue_steps(h, std::min(k, left));
}

int sim_sync(sim_t *h)
{
    int rc = check_handle(h);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        h->failed = true;
        return fail(SIM_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
    return SIM_OK;
}

int sim_query(sim_t *h)
{
    int rc = check_handle(h);
    if (rc) return rc;
    const hipError_t e = hipStreamQuery(h->stream);
    if (e == hipSuccess) return SIM_OK;
    if (e == hipErrorNotReady) return SIM_BUSY;
    h->failed = true;
    return fail(SIM_EDEVICE, std::string("hipStreamQuery: ") + hipGetErrorString(e));
}

int sim_member_info(sim_t *h, int32_t index, int64_t *n, int64_t *step, int64_t *n_steps)
{
    int rc = check_handle(h);
    if (rc) return rc;
    rc = check_member_index(h, index);
    if (rc) return rc;
    const Member &m = h->members[index];
    if (n) *n = m.n;
    if (step) *step = m.step_host;
    if (n_steps) *n_steps = m.seg.n_steps;
    return SIM_OK;
}

int sim_member_read_response(sim_t *h, int32_t index, int64_t first, int64_t count, double *q_diff)
{
    int rc = check_handle(h);
    if (rc) return rc;
    rc = check_member_index(h, index);
    if (rc) return rc;
    const Member &m = h->members[index];
    if (count == 0) return SIM_OK;
    if (!q_diff || count < 0 || first < m.start_step || first + count > m.step_host)
        return fail(SIM_ERANGE, "response range not computed");
    rc = sim_sync(h);
    if (rc) return rc;
    hipError_t e = hipMemcpy(q_diff, m.seg.qdiff + first, sizeof(double) * count, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return mark_failed(h, fail(SIM_EDEVICE, "copy of Q_diff failed"));
    return SIM_OK;
}

int sim_read_response(sim_t *h, int64_t first, int64_t count, double *q_diff)
{
    return sim_member_read_response(h, 0, first, count, q_diff);
}

int sim_member_read_state(sim_t *h, int32_t index, double *pos, double *vel, uint8_t *alive,
                          double *q_surface, int64_t *step)
{
    int rc = check_handle(h);
    if (rc) return rc;
    rc = check_member_index(h, index);
    if (rc) return rc;
    rc = sim_sync(h);
    if (rc) return rc;
    const Member &mb = h->members[index];
    Ctl ctl;
    if (hipMemcpy(&ctl, h->ctl + index, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess)
        return mark_failed(h, fail(SIM_EDEVICE, "copy of control block failed"));
    const int64_t n = mb.n;
    const size_t p0 = mb.seg.p0;
    const size_t na = ctl.n_cur, ng = ctl.n_dead;
    std::vector<double> a[6], g[6];
    std::vector<uint32_t> au(na), gu(ng);
    std::vector<uint8_t> ad(na);
    std::vector<PRec> ar(na);
    double *srcG[6] = {h->G.x, h->G.y, h->G.z, h->G.vx, h->G.vy, h->G.vz};
    for (int j = 0; j < 6; ++j) {
        g[j].resize(ng);
        if (ng && hipMemcpy(g[j].data(), srcG[j] + p0, 8 * ng, hipMemcpyDeviceToHost))
            return mark_failed(h, fail(SIM_EDEVICE, "state copy failed"));
    }
    if ((na && (hipMemcpy(ar.data(), h->A + p0, sizeof(PRec) * na, hipMemcpyDeviceToHost) ||
                hipMemcpy(ad.data(), h->dead + p0, na, hipMemcpyDeviceToHost))) ||
        (ng && hipMemcpy(gu.data(), h->G.uid + p0, 4 * ng, hipMemcpyDeviceToHost)))
        return mark_failed(h, fail(SIM_EDEVICE, "state copy failed"));
    for (int j = 0; j < 6; ++j) a[j].resize(na);
    for (size_t i = 0; i < na; ++i) {
        const PRec &r = ar[i];
        a[0][i] = r.x; a[1][i] = r.y; a[2][i] = r.z;
        a[3][i] = r.vx; a[4][i] = r.vy; a[5][i] = r.vz;
        au[i] = r.uid;
    }
    auto find = [&](uint32_t u) -> int64_t {
        auto it = std::lower_bound(mb.id_index.begin(), mb.id_index.end(),
                                   std::make_pair(u, (int64_t)-1));
        if (it == mb.id_index.end() || it->first != u) return -1;
        return it->second;
    };
    if (alive) std::memset(alive, 0, (size_t)n);
    auto put = [&](int64_t k, std::vector<double> *src, size_t i) {
        if (pos) for (int j = 0; j < 3; ++j) pos[3 * k + j] = src[j][i];
        if (vel) for (int j = 0; j < 3; ++j) vel[3 * k + j] = src[3 + j][i];
    };
    for (size_t i = 0; i < ng; ++i) {
        int64_t k = find(gu[i]);
        if (k < 0) return fail(SIM_EDEVICE, "unknown id in graveyard");
        put(k, g, i);
    }
    for (size_t i = 0; i < na; ++i) {
        if (ad[i]) continue;
        int64_t k = find(au[i]);
        if (k < 0) return fail(SIM_EDEVICE, "unknown id in state");
        put(k, a, i);
        if (alive) alive[k] = 1;
    }
    if (q_surface)
        *q_surface = (mb.q_surface0 + kQ * (double)(ctl.n_dead - ctl.n_dead_ion)) +
                     (double)ctl.n_dead_ion;
    if (step) *step = ctl.step;
    return SIM_OK;
}

int sim_member_counts(sim_t *h, int32_t index, int64_t *alive, int64_t *absorbed, int64_t *step)
{
    int rc = check_handle(h);
    if (rc) return rc;
    rc = check_member_index(h, index);
    if (rc) return rc;
    rc = sim_sync(h);
    if (rc) return rc;
    Ctl ctl;
    if (hipMemcpy(&ctl, h->ctl + index, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess)
        return mark_failed(h, fail(SIM_EDEVICE, "copy of control block failed"));
    if (alive) *alive = h->members[index].n - (int64_t)ctl.n_dead;
    if (absorbed) *absorbed = (int64_t)ctl.n_dead;
    if (step) *step = ctl.step;
    return SIM_OK;
}

int sim_read_state(sim_t *h, double *pos, double *vel, uint8_t *alive, double *q_surface,
                   int64_t *step)
{
    return sim_member_read_state(h, 0, pos, vel, alive, q_surface, step);
}

int sim_member_eval_field(sim_t *h, int32_t index, double *E)
{
    int rc = check_handle(h);
    if (rc) return rc;
    rc = check_member_index(h, index);
    if (rc) return rc;
    if (!E) return fail(SIM_EINVAL, "E is NULL");
    rc = launch_step(h, h->stream, true, nullptr);
    if (rc) return mark_failed(h, rc);
    rc = sim_sync(h);
    if (rc) return rc;
    const Member &mb = h->members[index];
    Ctl ctl;
    if (hipMemcpy(&ctl, h->ctl + index, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess)
        return mark_failed(h, fail(SIM_EDEVICE, "copy of control block failed"));
    const size_t nl = ctl.n_live, p0 = mb.seg.p0;
    std::vector<double> e(3 * nl);
    std::vector<uint32_t> u(nl);
    if (nl && (hipMemcpy(e.data(), h->Eout + 3 * p0, 8 * 3 * nl, hipMemcpyDeviceToHost) ||
               hipMemcpy(u.data(), h->Eid + p0, 4 * nl, hipMemcpyDeviceToHost)))
        return mark_failed(h, fail(SIM_EDEVICE, "field copy failed"));
    std::memset(E, 0, sizeof(double) * 3 * (size_t)mb.n);
    for (size_t i = 0; i < nl; ++i) {
        auto it = std::lower_bound(mb.id_index.begin(), mb.id_index.end(),
                                   std::make_pair(u[i], (int64_t)-1));
        if (it == mb.id_index.end() || it->first != u[i]) return fail(SIM_EDEVICE, "unknown id");
        for (int j = 0; j < 3; ++j) E[3 * it->second + j] = e[3 * i + j];
    }
    return SIM_OK;
}

int sim_eval_field(sim_t *h, double *E) { return sim_member_eval_field(h, 0, E); }

int64_t sim_eval_field_static_bytes(const sim_params *p, int64_t n)
{
    std::string why;
    if (!check_common(p, &why)) return fail(SIM_EINVAL, why);
    if (n <= 0 || n > 0x7fffffffLL) return fail(SIM_EINVAL, "n must be in [1, 2^31)");
    return footprint(p, slots_for(n), 1, member_shape(n, tuning_of(p)).nc, member_bytes(1, 0));
}

int sim_eval_field_static(const sim_params *p, int64_t n, const double *pos, double q_surface,
                          double u_asy, double *E, void *hip_stream)
{
    std::string why;
    if (!check_common(p, &why)) return fail(SIM_EINVAL, why);
    if (n <= 0 || n > 0x7fffffffLL) return fail(SIM_EINVAL, "n must be in [1, 2^31)");
    if (!pos || !E) return fail(SIM_EINVAL, "pos and E are required");
    if (!std::isfinite(q_surface) || !std::isfinite(u_asy))
        return fail(SIM_EINVAL, "q_surface and u_asy must be finite");
    sim_member m = member_from_params(p, n, nullptr, nullptr, nullptr, nullptr, 1, 0);
    if (!check_member_scalars(&m, &why)) return fail(SIM_EINVAL, why);
    const MemberShape sh = member_shape(n, tuning_of(p));
    // the same layout as sim_create's for these particles
    sim h;
    if (!make_layout(p, slots_for(n), 1, sh.nc, &h.lo, &why)) return fail(SIM_EINVAL, why);
    h.prm = *p;
    Alloc al;
    plan_alloc(&h, al, member_bytes(1, 0));
    if (al.total() > kScratchBytes)
        return fail(SIM_ENOMEM, "evaluation needs " + std::to_string(al.total()) +
                                    " B of working memory, more than the static buffer's " +
                                    std::to_string(kScratchBytes) + " B");
    void *base = nullptr;
    if (int rc = scratch_address(&base)) return rc;
    carve(al, base);
    HostTables ht;
    if (int rc = make_host_tables(*p, h.lo, &ht)) return rc;
    bind_device_tables(&h);
    h.ext.n_tiles = (int)sh.nt;
    h.ext.n_chunks = (int)sh.nc;
    h.ext.nb = (int)sh.nb;
    h.ext.nb_blocks = ((int)sh.nb + kScanPerBlock - 1) / kScanPerBlock;
    h.ext.n_members = 1;
    Seg sg{};
    sg.p0 = 0;
    sg.cap = sh.ng * kGroupSlots;
    sg.t0 = 0;
    sg.nt = sh.nt;
    sg.g0 = 0;
    sg.ng = sh.ng;
    sg.c0 = 0;
    sg.nc = sh.nc;
    sg.cl = sh.cl;
    sg.b0 = 0;
    sg.nb = sh.nb;
    sg.inv_vol = 1.0 / (p->r_out * p->r_out * p->r_out - 1.0);
    sg.ntilde = p->ntilde;
    sg.inv_ntilde = 1.0 / p->ntilde;
    sg.ion_density = p->ion_density;
    sg.q_surface0 = q_surface;
    sg.dt = p->dt;
    sg.r_out = p->r_out;
    sg.seed = p->seed;
    sg.probe_bc = p->probe_bc;
    sg.wall_bc = p->wall_bc;
    sg.n_steps = 1;
    sg.u_asy = reinterpret_cast<double *>(h.mdata);
    sg.qdiff = reinterpret_cast<double *>(h.mdata + kPoolUnit);
    sg.near_w = near_width(h.lo.tu, h.lo.fp32, h.lo.L, n);
    sg.used = 1;
    Ctl ct{};
    ct.step = 0;
    ct.n_cur = (uint32_t)n;
    ct.n_live = (uint32_t)n;
    ct.q_surface = q_surface;
    ct.keys_for = -1;
    hipStream_t s = (hipStream_t)hip_stream;
    const unsigned gSet = (unsigned)std::min<int64_t>(((int64_t)sh.nt * kWave + kBlock - 1) / kBlock, 4096);
    const unsigned gN = (unsigned)((n + kBlock - 1) / kBlock);
    k_static_setup<<<gSet, kBlock, 0, s>>>(sg, ct, h.seg, h.ctl, h.tile_member, h.chunk_member,
                                           h.dead, h.hist, const_cast<double *>(sg.u_asy), u_asy,
                                           (int)sh.nt, (int)sh.nc, h.lo.nb);
    k_static_pack<<<gN, kBlock, 0, s>>>(pos, (uint32_t)n, h.A);
    HIP_TRY(hipMemcpyAsync(h.tables, ht.tab.data(), sizeof(double) * ht.tab.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h.chl, ht.chl.data(), sizeof(int) * ht.chl.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h.chn, ht.chn.data(), sizeof(double) * ht.chn.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h.chg, ht.chg.data(), sizeof(double) * ht.chg.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h.tables32, ht.tab32.data(), sizeof(float) * ht.tab32.size(),
                           hipMemcpyHostToDevice, s));
    if (int rc = launch_step(&h, s, true, nullptr)) return rc;
    k_static_unpack<<<gN, kBlock, 0, s>>>(h.Eout, h.Eid, (uint32_t)n, E);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return fail(SIM_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
    // the host tables above are the copies' sources: done before they go
    HIP_TRY(hipStreamSynchronize(s));
    return SIM_OK;
}

int sim_profile(sim_t *h, int64_t k, double *kernel_ms, int32_t n_kernels)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (k <= 0 || !kernel_ms) return fail(SIM_EINVAL, "k must be > 0 and kernel_ms non-NULL");
    for (const Member &m : h->members)
        if (m.used && m.step_host + k > m.seg.n_steps) return fail(SIM_ERANGE, "steps beyond n_steps");
    hipEvent_t ev[KN_COUNT + 1];
    for (int i = 0; i <= KN_COUNT; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) return fail(SIM_EDEVICE, "hipEventCreate failed");
    std::vector<double> acc(KN_COUNT, 0.0);
    for (int64_t s = 0; s < k && rc == SIM_OK; ++s) {
        rc = launch_step(h, h->stream, false, ev);
        if (rc == SIM_OK && hipEventSynchronize(ev[KN_COUNT]) != hipSuccess)
            rc = fail(SIM_EDEVICE, "event sync failed");
        for (int i = 0; i < KN_COUNT && rc == SIM_OK; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) acc[i] += ms;
        }
        if (rc == SIM_OK)
            for (Member &m : h->members)
                if (m.used) m.step_host += 1;
    }
    for (int i = 0; i <= KN_COUNT; ++i) (void)hipEventDestroy(ev[i]);
    if (rc) return mark_failed(h, rc);
    for (int i = 0; i < KN_COUNT && i < n_kernels; ++i) kernel_ms[i] = acc[i] / (double)k;
    return SIM_OK;
}

int32_t sim_num_kernels(void) { return KN_COUNT; }

const char *sim_kernel_name(int32_t i)
{
    if (i < 0 || i >= KN_COUNT) return "";
    return kKernelNames[i];
}

int sim_info(sim_t *h, int64_t *n, int32_t *tile, int32_t *channels)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (n) *n = h->members.empty() || !h->members[0].used ? 0 : h->members[0].n;
    if (tile) *tile = kWave;
    if (channels) *channels = h->lo.C;
    return SIM_OK;
}

void sim_destroy(sim_t *h)
{
    if (!h) return;
    release(h);
    delete h;
}

const char *sim_strerror(int status)
{
    switch (status) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument";
    case SIM_ENOMEM: return "out of memory or over the memory limit";
    case SIM_ERANGE: return "index out of range";
    case SIM_ESTATE: return "invalid or failed handle";
    case SIM_EDEVICE: return "HIP runtime error";
    case SIM_BUSY: return "work still running";
    default: return "unknown status";
    }
}

const char *sim_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
