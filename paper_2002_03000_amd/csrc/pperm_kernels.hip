// gfx950 kernels of parallel flatPERM (Campbell & Janse van Rensburg,
// "Parallel PERM"): Rosenbluth growth with a_+ occupancy scans (Sec. 1,
// eqns (1)-(2)), flatPERM prune/enrich against the running averages (Sec. 2,
// eqn (6)), accumulation of the sample sums (eqn (4)), and the merge of the
// per-sequence sums into the pooled sums of Algorithm 2 (Sec. 3, Fig. 1).
//
// Execution model.  The default growth kernel (batch_kernel) is persistent:
// one 64-lane wavefront takes one (problem, sequence) item at a time from a
// device queue and runs that sequence's tours; every walk quantity is uniform
// over the wave, and the lanes split the parallel parts of a step:
//   - the occupancy scan: lane (dir, off) reads slot home(dir)+off+W*round of
//     the walk's open-addressing table, so the 2d neighbours and W consecutive
//     probe positions per neighbour are looked up in one LDS instruction and
//     resolved with two wave ballots;
//   - the random numbers: lane i computes the Philox4x32-10 block of event
//     k0+i, so one pass of the (quarter-rate) multiplies serves 64 events;
//   - the LIFO deletion of abandoned sites after a backtrack.
// The walk's occupancy table (packed coordinates, linear probing, restored
// exactly by LIFO deletion through remembered slot ids), the slot ids and the
// sequence's own per-length sums live in LDS (the sums in global memory for
// long walks); the 64 most recent pending copies live in the lanes of a few
// vector registers; the pooled sums are read with scalar loads.  A second kernel
// (run_kernel) packs 64/TS walks into a wave as teams of TS lanes.
//
// Determinism.  Every floating-point decision uses the same IEEE operations
// in the same order as the reading of the method these kernels implement
// (no contraction: the library is built with -ffp-contract=off), and the
// random numbers are a pure function of (seed, sequence, tour, event).  The
// launch shape therefore never changes a result.
#include <mutex>

#include "pperm_internal.h"

namespace pperm {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, Weyl key schedule.
// ---------------------------------------------------------------------------
constexpr uint32_t PHX_M0 = 0xD2511F53u;
constexpr uint32_t PHX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHX_W0 = 0x9E3779B9u;
constexpr uint32_t PHX_W1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = PHX_M0 * c.x, hi0 = __umulhi(PHX_M0, c.x);
        const uint32_t lo1 = PHX_M1 * c.z, hi1 = __umulhi(PHX_M1, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += PHX_W0;
        k1 += PHX_W1;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Extended-range weights: x = m * 2^e, m in [0.5, 1) (m = 0, e = 0 for zero).
// Every operation is the correctly rounded result of the exact operation on
// the represented values (frexp and ldexp by at most 63 binades are exact),
// so weights of any size are carried without underflow or overflow.
// ---------------------------------------------------------------------------
struct XF {
    double m;
    int e;
};

__device__ __forceinline__ XF xf_norm(double x, int e) {
    const double m = __builtin_amdgcn_frexp_mant(x);
    const int k = __builtin_amdgcn_frexp_exp(x);
    XF r;
    r.m = m;
    r.e = (m == 0.0) ? 0 : e + k;
    return r;
}

// Written with selects only (no branches): the operand with the larger
// exponent keeps its scale, the other is shifted onto it.  The shift is exact
// while the shifted mantissa stays normal; once it has moved 54 or more
// binades it is below half an ulp of the kept mantissa (which lies in
// [0.5, 1)), so the rounded sum is the kept mantissa whatever it became --
// the same as dropping it, which is how the exact operation is usually
// written (a shift beyond 63 binades is dropped).
__device__ __forceinline__ XF xf_add(XF a, XF b) {
    const bool sw = a.e < b.e;
    const double hm = sw ? b.m : a.m;
    const int he = sw ? b.e : a.e;
    const double lm = sw ? a.m : b.m;
    const int le = sw ? a.e : b.e;
    const int d = he - le;
    const double ls = ldexp(lm, -d);
    XF r = xf_norm(hm + ls, he);
    // zero operands (field by field, so that no struct is selected by address)
    const bool az = (a.m == 0.0), bz = (b.m == 0.0);
    r.m = az ? b.m : (bz ? a.m : r.m);
    r.e = az ? b.e : (bz ? a.e : r.e);
    return r;
}

__device__ __forceinline__ XF xf_mul(XF a, double k) { return xf_norm(a.m * k, a.e); }
__device__ __forceinline__ XF xf_div(XF a, double k) { return xf_norm(a.m / k, a.e); }

// a / b as an ordinary double, exponent gap clamped to [-1000, 1000].
__device__ __forceinline__ double xf_ratio(XF a, XF b) {
    const int d = a.e - b.e;
    const int dc = d < -1000 ? -1000 : (d > 1000 ? 1000 : d);
    double r = ldexp(a.m / b.m, dc);
    r = (d > 1000) ? 0x1p1000 : r;
    r = (d < -1000 || a.m == 0.0) ? 0.0 : r;
    return r;
}

// The same operations where an operand is known to be nonzero (every walk
// weight and every sum that includes one): they give the same result as the
// general ones on such operands, with the zero cases left out.
__device__ __forceinline__ XF xf_norm_nz(double x, int e) {
    XF r;
    r.m = __builtin_amdgcn_frexp_mant(x);
    r.e = e + __builtin_amdgcn_frexp_exp(x);
    return r;
}

// a + b for b != 0: both mantissas are brought to the larger exponent (the
// larger operand's by an exact shift of 0, the other's as in xf_add) and
// added, so no operand swap is needed.  A zero a counts as having the
// smallest exponent: shifted away, its mantissa 0 leaves exactly b.
__device__ __forceinline__ XF xf_add_nz(XF a, XF b) {
    const int ae = (a.m == 0.0) ? -0x40000000 : a.e;
    const int he = ae > b.e ? ae : b.e;
    return xf_norm_nz(ldexp(a.m, ae - he) + ldexp(b.m, b.e - he), he);
}

// x / y, correctly rounded, for operands whose quotient and reciprocal are
// far from the ends of the FP64 range: x in [0.5, 1) and y in [0.5, 2^34]
// here (a mantissa, or a mantissa over an integer below 2^34).  Markstein's
// method: the hardware reciprocal refined by two Newton-Raphson steps with
// fused multiply-adds, the quotient x * y, and one correction with the exact
// residual x - y q.  It is the general IEEE division sequence without its
// operand scaling and special-case fix-up, which leave such operands and
// their quotient unchanged.
__device__ __forceinline__ double div_normal(double x, double y) {
    double r = __builtin_amdgcn_rcp(y);
    double e = __builtin_fma(-y, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-y, r, 1.0);
    r = __builtin_fma(r, e, r);
    const double q = x * r;
    const double res = __builtin_fma(-y, q, x);
    return __builtin_fma(res, r, q);
}

__device__ __forceinline__ XF xf_mul_nz(XF a, double k) { return xf_norm_nz(a.m * k, a.e); }
// a / k for an integer 2 <= k < 2^34
__device__ __forceinline__ XF xf_div_nz(XF a, double k) { return xf_norm_nz(div_normal(a.m, k), a.e); }

// a / b for a, b != 0 whose ratio is below 2^34 (a decision's W * seen over a
// sum that includes N copies of W, see walk_sequence): the exponent gap is at
// most 35, so of the general clamp to [-1000, 1000] only the lower end can act.
__device__ __forceinline__ double xf_ratio_nz(XF a, XF b) {
    const int d = a.e - b.e;
    const double r = ldexp(div_normal(a.m, b.m), d < -1000 ? -1000 : d);
    return (d < -1000) ? 0.0 : r;
}

__device__ __forceinline__ XF xf_of(const SumRec& r) { return XF{r.m, r.e}; }

// ---------------------------------------------------------------------------
// Lattice: packed int16 coordinates (offset by 2^15 so that key 0 never
// occurs and marks an empty slot), direction order +x,-x,+y,-y,+z,-z.
// ---------------------------------------------------------------------------
template <int D> struct Lat;
template <> struct Lat<2> {
    using Key = uint32_t;
    static constexpr int D = 2;
    static constexpr int DP = 4;  // direction lanes per probe window
    __device__ static Key origin() { return pack(0, 0, 0); }
    // neighbour key = end key + delta(dir): no field ever carries, every
    // coordinate stays within +-n_max < 2^15 of its 2^15 offset
    __device__ static Key delta(int dir) {
        if (dir >= 4) return 0u;
        const Key mag = (Key)1 << (16 * (dir >> 1));
        return (dir & 1) ? (Key)((Key)0 - mag) : mag;
    }
    __device__ static Key next(Key k, Key d) { return k + d; }
    __device__ static Key pack(int x, int y, int) {
        return (uint32_t)(x + 32768) | ((uint32_t)(y + 32768) << 16);
    }
    __device__ static void unpack(Key k, int& x, int& y, int& z) {
        x = (int)(k & 0xFFFFu) - 32768;
        y = (int)(k >> 16) - 32768;
        z = 0;
    }
    __device__ static uint32_t hash(Key k) { return k * 0x9E3779B1u; }
};
template <> struct Lat<3> {
    using Key = uint64_t;
    static constexpr int D = 3;
    static constexpr int DP = 8;
    __device__ static Key origin() { return pack(0, 0, 0); }
    __device__ static Key delta(int dir) {
        if (dir >= 6) return 0u;
        const Key mag = (Key)1 << (16 * (dir >> 1));
        return (dir & 1) ? (Key)((Key)0 - mag) : mag;
    }
    __device__ static Key next(Key k, Key d) { return k + d; }
    __device__ static Key pack(int x, int y, int z) {
        return (uint64_t)(uint32_t)(x + 32768) | ((uint64_t)(uint32_t)(y + 32768) << 16) |
               ((uint64_t)(uint32_t)(z + 32768) << 32);
    }
    __device__ static void unpack(Key k, int& x, int& y, int& z) {
        x = (int)(k & 0xFFFFu) - 32768;
        y = (int)((k >> 16) & 0xFFFFu) - 32768;
        z = (int)((k >> 32) & 0xFFFFu) - 32768;
    }
    __device__ static uint32_t hash(Key k) {
        return (uint32_t)k * 0x9E3779B1u + (uint32_t)(k >> 32) * 0x85EBCA77u;
    }
};

// The cubic lattice for walks of at most COMPACT3_MAX_N steps, with 32-bit
// keys: each coordinate modulo 1024 in a 10-bit field (x in bits 0-9, y in
// 11-20, z in 22-31) with a zero guard bit between fields, the origin at 512
// in every field.  Any two sites of one walk, and a site of the walk and a
// neighbour of its end, differ by at most n_max + 1 <= 1023 in every
// coordinate, so their keys differ; key 0 would need |x| + |y| + |z| >= 1536.
// A neighbour's key is the end's key plus a per-direction offset (-1 is +1023
// in the field), with the carry out of a field dropped at its guard bit.
struct Lat3c {
    static constexpr int D = 3;
    using Key = uint32_t;
    static constexpr uint32_t GUARD = (1u << 10) | (1u << 21);
    __device__ static Key origin() { return 512u | (512u << 11) | (512u << 22); }
    // offset of direction dir (+x, -x, +y, -y, +z, -z); 0 past the six
    __device__ static Key delta(int dir) {
        if (dir >= 6) return 0u;
        const uint32_t sh = 11u * (uint32_t)(dir >> 1);
        return (dir & 1) ? (1023u << sh) : (1u << sh);
    }
    __device__ static Key next(Key k, Key d) { return (k + d) & ~GUARD; }
    __device__ static uint32_t hash(Key k) { return k * 0x9E3779B1u; }
};

// The lattice (key format) a walker instance uses: packed int16 coordinates,
// or the compact cubic keys above.
template <int D, bool CK> struct LatOf { using T = Lat<D>; };
template <> struct LatOf<3, true> { using T = Lat3c; };

__device__ __forceinline__ int dir_dx(int d) { return (d == 0) - (d == 1); }
__device__ __forceinline__ int dir_dy(int d) { return (d == 2) - (d == 3); }
__device__ __forceinline__ int dir_dz(int d) { return (d == 4) - (d == 5); }

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Team phases.
enum : int { PH_NEED_SEQ = 0, PH_NEED_TOUR = 1, PH_NEED_BT = 2, PH_AT_NODE = 3, PH_DONE = 4,
             PH_ABORT = 5 };

// Trajectory digest of a sequence (instrumentation, not part of the method):
// FNV-1a 32 over one byte per growth step, dir | a_+ << 3, kept zero-extended
// in a 64-bit statistics word.
constexpr uint32_t FNV_OFFSET = 2166136261u;
constexpr uint32_t FNV_PRIME = 16777619u;

// Bits 0, DP, 2*DP, ... (W of them): the lanes of one direction in a team.
template <int DP, int W>
__device__ __forceinline__ uint64_t dir_rep() {
    uint64_t r = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) r |= 1ull << (j * DP);
    return r;
}

// Fold a team-local lane mask (TS bits) onto direction bits (DP bits).
template <int TS, int DP>
__device__ __forceinline__ uint32_t fold_dirs(uint64_t x) {
#pragma unroll
    for (int s = TS / 2; s >= DP; s /= 2) x |= x >> s;
    return (uint32_t)(x & ((1u << DP) - 1u));
}

template <int D, int TS>
__global__ void __launch_bounds__(64) run_kernel(RunArgs A) {
    using L_ = Lat<D>;
    using Key = typename L_::Key;
    constexpr int DP = L_::DP;
    static_assert(TS >= DP && TS <= 64 && (TS & (TS - 1)) == 0, "team size");
    constexpr int W = TS / DP;          // probe positions per direction per round
    constexpr int TPW = 64 / TS;        // teams per wave

    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = (int)threadIdx.x;
    const int lt = lane & (TS - 1);
    const int tbase = lane & ~(TS - 1);
    const int tiw = lane / TS;
    const uint32_t team_slot = blockIdx.x * TPW + tiw;

    Key* table = reinterpret_cast<Key*>(lds + (size_t)tiw * A.lds_team_bytes);
    uint16_t* sid = reinterpret_cast<uint16_t*>(lds + (size_t)tiw * A.lds_team_bytes +
                                                (sizeof(Key) << A.slots_log2));
    const uint32_t S = 1u << A.slots_log2;
    const uint32_t smask = S - 1u;
    const uint32_t hshift = 32u - A.slots_log2;

    // probe-lane role
    const int pdir = lt % DP;
    const int poff = lt / DP;
    const bool pvalid = pdir < 2 * D;
    const int pdx = dir_dx(pdir), pdy = dir_dy(pdir), pdz = dir_dz(pdir);
    const uint64_t same_dir = dir_rep<DP, W>() << (tbase + pdir);
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const uint64_t same_dir_below = same_dir & below;

    const uint32_t n_max = A.n_max;
    const uint32_t row = A.row;
    const bool shared_mode = (A.mode == MODE_SHARED);
    const bool control_mode = (A.mode != MODE_ROSENBLUTH);
    // in Algorithm 2 a sequence's own epoch data stands for the pool's: weight N
    const double pool = shared_mode ? (double)A.N : 1.0;
    const uint64_t pool_u = shared_mode ? (uint64_t)A.N : 1ull;
    const uint32_t cap = A.step_cap;

    // empty table with the origin in it; slot id of site 0
    for (uint32_t i = (uint32_t)lt; i < S; i += TS) table[i] = (Key)0;
    wave_fence();
    const Key origin_key = L_::pack(0, 0, 0);
    if (lt == 0) {
        const uint32_t h = L_::hash(origin_key) >> hshift;
        table[h] = origin_key;
        sid[0] = (uint16_t)h;
    }
    wave_fence();

    StackEntry* stk = A.stack + (size_t)team_slot * n_max;

    // ---- team state (identical in every lane of a team) ----
    int phase = PH_NEED_SEQ;
    uint32_t s = 0, tours_left = 0, m = 0;
    uint64_t t = 0, tt = 0;
    SumRec rec0 = {0.0, 0, 0u};           // L[s][0]: one record per tour
    const SumRec* Grow = A.G;
    uint64_t MGs = shared_mode ? A.MG[0] : 0;
    uint64_t st_steps = 0, st_events = 0, st_enrich = 0, st_copies = 0, st_prunes = 0,
             st_traps = 0, st_tours = 0, st_maxd = 0, st_digest = 0, st_capped = 0;
    uint32_t steps_call = 0;

    uint32_t n = 0;
    XF w = {0.5, 1};
    int ex = 0, ey = 0, ez = 0;
    bool control = false;
    uint64_t k = 0, kb = 0;
    bool stale = true;
    uint4 rb = make_uint4(0, 0, 0, 0);

    uint32_t sp = 0, top_n = 0, top_rem = 0;
    XF top_w = {0.0, 0};

    SumRec Lp = {0.0, 0, 0u}, Gp = {0.0, 0, 0u};   // records of length n + 1 (prefetched)
    XF Lc = {0.0, 0}, Gc = {0.0, 0};               // sums at length n after its record

    for (;;) {
        // ---------------- (1) acquire a sequence ----------------
        const bool need_seq = (phase == PH_NEED_SEQ);
        uint32_t got = 0xFFFFFFFFu;
        if (need_seq && lt == 0) got = atomicAdd(&A.ctrl[CTRL_QUEUE], 1u);
        got = __shfl(got, tbase, 64);
        if (need_seq) {
            if (got < A.N) {
                s = got;
                const size_t rb0 = (size_t)s * row;
                t = A.t[s];
                m = A.m[s];
                rec0 = A.L[rb0];
                const uint64_t* sr = A.stats + (size_t)s * STATS_WORDS;
                st_steps = sr[ST_STEPS]; st_events = sr[ST_EVENTS]; st_enrich = sr[ST_ENRICH];
                st_copies = sr[ST_COPIES]; st_prunes = sr[ST_PRUNES]; st_traps = sr[ST_TRAPS];
                st_tours = sr[ST_TOURS]; st_maxd = sr[ST_MAXDEPTH]; st_digest = sr[ST_DIGEST];
                st_capped = sr[ST_CAPPED];
                if (!shared_mode) {
                    Grow = A.G + rb0;
                    MGs = A.MG[s];
                }
                tours_left = A.tours;
                steps_call = 0;
                phase = PH_NEED_TOUR;
            } else {
                phase = PH_DONE;
            }
        }
        if (__ballot(phase != PH_DONE) == 0ull) break;

        SumRec* Lrow = A.L + (size_t)s * row;

        // ---------------- (2) backtrack / end of tour ----------------
        if (phase == PH_NEED_BT || phase == PH_ABORT) {
            const bool abort = (phase == PH_ABORT);
            const bool tour_end = abort || sp == 0;
            uint32_t rn = 0;
            if (!tour_end) {
                rn = top_n;
                w = top_w;
                top_rem -= 1;
                if (top_rem == 0) {
                    sp -= 1;
                    if (sp > 0) {
                        const StackEntry e = stk[sp - 1];
                        top_n = e.n;
                        top_rem = e.remaining;
                        top_w = XF{e.m, e.e};
                    }
                }
            }
            // LIFO deletion of sites rn+1..n restores the table exactly
            for (uint32_t i = rn + 1 + (uint32_t)lt; i <= n; i += TS) table[sid[i]] = (Key)0;
            if (!tour_end) {
                const Key ek = table[sid[rn]];
                L_::unpack(ek, ex, ey, ez);
                n = rn;
                control = false;
                phase = PH_AT_NODE;
                Lp = Lrow[n + 1];
                Gp = Grow[n + 1];
            } else {
                n = 0;
                ex = ey = ez = 0;
                sp = 0;
                if (abort) {
                    st_capped = 1;
                    tours_left = 0;
                    if (lt == 0) atomicOr(&A.ctrl[CTRL_ERR], ERR_CAP);
                } else {
                    tours_left -= 1;
                }
                if (tours_left > 0) {
                    phase = PH_NEED_TOUR;
                } else {
                    if (lt == 0) {
                        const size_t rb0 = (size_t)s * row;
                        A.L[rb0] = rec0;
                        A.t[s] = t;
                        A.m[s] = m;
                        uint64_t* sr = A.stats + (size_t)s * STATS_WORDS;
                        sr[ST_STEPS] = st_steps; sr[ST_EVENTS] = st_events; sr[ST_ENRICH] = st_enrich;
                        sr[ST_COPIES] = st_copies; sr[ST_PRUNES] = st_prunes; sr[ST_TRAPS] = st_traps;
                        sr[ST_TOURS] = st_tours; sr[ST_MAXDEPTH] = st_maxd; sr[ST_DIGEST] = st_digest;
                        sr[ST_CAPPED] = st_capped;
                    }
                    phase = PH_NEED_SEQ;
                }
            }
        }

        // ---------------- (3) start of a tour ----------------
        if (phase == PH_NEED_TOUR) {
            tt = t;
            t += 1;
            m += 1;
            st_tours += 1;
            w = XF{0.5, 1};                       // W_0 = 1
            {
                const XF r0 = xf_add(xf_of(rec0), w);
                rec0.m = r0.m;
                rec0.e = r0.e;
                rec0.h += 1u;
            }
            k = 0;
            stale = true;
            n = 0;
            ex = ey = ez = 0;
            control = false;
            phase = PH_AT_NODE;
            Lp = Lrow[1];
            Gp = Grow[1];
        }
        wave_fence();

        // ---------------- (4) occupancy scan at the endpoint ----------------
        const bool probing = (phase == PH_AT_NODE);
        const Key nk = L_::pack(ex + pdx, ey + pdy, ez + pdz);
        const uint32_t home = L_::hash(nk) >> hshift;
        bool open = probing && pvalid;
        uint32_t freem = 0;
        int my_ins = -1;
        uint32_t pos = home + (uint32_t)poff;
        for (;;) {
            if (__ballot(open) == 0ull) break;
            bool hit = false, emp = false;
            uint32_t slot = 0;
            if (open) {
                slot = pos & smask;
                const Key v = table[slot];
                hit = (v == nk);
                emp = (v == (Key)0);
            }
            const bool res = hit || emp;
            const uint64_t bres = __ballot(res);
            const bool first = res && ((bres & same_dir_below) == 0ull);
            const uint64_t bfe = __ballot(first && emp);
            const uint64_t bfr = __ballot(first);
            const uint64_t tmaskl = (TS == 64) ? ~0ull : ((1ull << TS) - 1ull);
            freem |= fold_dirs<TS, DP>((bfe >> tbase) & tmaskl);
            const uint32_t done_dirs = fold_dirs<TS, DP>((bfr >> tbase) & tmaskl);
            if (first && emp) my_ins = (int)slot;
            if ((done_dirs >> pdir) & 1u) open = false;
            pos += W;
        }
        const uint32_t a = (uint32_t)__popc(freem);
        if (probing && a == 0) {
            st_traps += 1;
            phase = PH_NEED_BT;
        }

        // ---------------- (5) random blocks ----------------
        const bool growing = (phase == PH_AT_NODE);
        if (__ballot(growing && (stale || (k - kb) >= (uint64_t)TS)) != 0ull) {
            kb = k;
            stale = false;
            const uint64_t kk = kb + (uint64_t)lt;
            rb = philox10(make_uint4((uint32_t)kk, (uint32_t)(kk >> 32), (uint32_t)tt, s), A.key0,
                          A.key1);
        }
        const int src = tbase + (int)((uint32_t)(k - kb) & (uint32_t)(TS - 1));
        const uint32_t B0 = __shfl(rb.x, src, 64);
        const uint32_t B1 = __shfl(rb.y, src, 64);
        const uint32_t B2 = __shfl(rb.z, src, 64);

        // ---------------- (6) decision, growth, record ----------------
        if (growing) {
            k += 1;
            st_events += 1;
            bool pruned = false;
            if (control) {
                // eqn (6): r = W / [W_n], [W_n] = sum / seen with the sequence's
                // own epoch data weighted N; evaluated as (W * seen) / sum
                const XF sum = xf_add(Gc, xf_mul(Lc, pool));
                const double seen = (double)(MGs + pool_u * (uint64_t)m);
                const double r = xf_ratio(xf_mul(w, seen), sum);
                const double u = ((double)(B1 >> 5) * 67108864.0 + (double)(B2 >> 6)) *
                                 (1.0 / 9007199254740992.0);
                if (r >= 1.0) {
                    const double f = floor(r);
                    double c;
                    if (r != f && u < (f + 1.0) - r) c = f;
                    else c = (r == f) ? f : f + 1.0;
                    w = xf_div(w, c);
                    if (c > 1.0) {
                        const uint32_t ci = (uint32_t)c;
                        if (sp > 0) {
                            // every lane of the team stores (and later reloads) the
                            // entry, so each lane only ever reads its own writes
                            StackEntry e;
                            e.n = top_n;
                            e.remaining = top_rem;
                            e.e = top_w.e;
                            e.pad0 = 0u;
                            e.m = top_w.m;
                            e.key = 0ull;
                            stk[sp - 1] = e;
                        }
                        top_n = n;
                        top_rem = ci - 1u;
                        top_w = w;
                        sp += 1;
                        if ((uint64_t)sp > st_maxd) st_maxd = sp;
                        st_enrich += 1;
                        st_copies += (uint64_t)(ci - 1u);
                    }
                } else {
                    // a survivor takes W / r, the running average itself
                    if (u < r) w = xf_div(sum, seen);
                    else pruned = true;
                }
            }
            if (pruned) {
                st_prunes += 1;
                phase = PH_NEED_BT;
            } else {
                const uint32_t j = __umulhi(B0, a);
                uint32_t mm = freem;
                for (uint32_t i = 0; i < j; ++i) mm &= mm - 1u;
                const int dir = __ffs(mm) - 1;
                st_digest = (uint64_t)(((uint32_t)st_digest ^ ((uint32_t)dir | (a << 3))) * FNV_PRIME);
                if (my_ins >= 0 && pdir == dir) {
                    table[my_ins] = nk;
                    sid[n + 1] = (uint16_t)my_ins;
                }
                ex += dir_dx(dir);
                ey += dir_dy(dir);
                ez += dir_dz(dir);
                w = xf_mul(w, (double)a);      // W *= a_+, eqn (2)
                if (w.e > EXP_LIMIT || w.e < -EXP_LIMIT) {
                    if (lt == 0) atomicOr(&A.ctrl[CTRL_ERR], ERR_RANGE);
                }
                n += 1;
                st_steps += 1;
                steps_call += 1;
                // arrival: record into the running sums (eqn (4))
                const XF Lnew = xf_add(xf_of(Lp), w);
                SumRec nr;
                nr.m = Lnew.m;
                nr.e = Lnew.e;
                nr.h = Lp.h + 1u;
                Lrow[n] = nr;
                Lc = Lnew;
                Gc = xf_of(Gp);
                if (cap != 0u && steps_call >= cap) {
                    phase = PH_ABORT;
                } else if (n == n_max) {
                    phase = PH_NEED_BT;
                } else {
                    control = control_mode;
                    Lp = Lrow[n + 1];
                    Gp = Grow[n + 1];
                }
            }
        }
        wave_fence();
    }
}

// ---------------------------------------------------------------------------
// Wave-per-walk growth kernel.  One 64-lane wavefront owns one walk, so every
// quantity of the walk is uniform across the wave and every branch is a
// scalar branch; the lanes only split the occupancy scan (lane = dir * W + off
// reads probe position off of direction dir), the Philox blocks (lane i holds
// the block of event kb + i, fetched with readlane) and the LIFO deletions.
// The sequence's own per-length sums live in LDS while its tours run (no
// global round trip on the record / decision path), the pooled sums are read
// with scalar loads, and each pending-copy entry carries its endpoint site, so
// a backtrack needs no table lookup to restore the walk's end.
// ---------------------------------------------------------------------------
// OR of v over aligned groups of G lanes (G = 8 or 16), every lane of a group
// receiving the group's OR: DPP quad permutes, then half-row and row mirrors.
template <int G>
__device__ __forceinline__ uint32_t group_or(uint32_t v) {
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if (G == 16) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    return v;
}

__device__ __forceinline__ uint32_t ufirst(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int ufirst_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t ufirst64(uint64_t v) {
    return ((uint64_t)ufirst((uint32_t)(v >> 32)) << 32) | (uint64_t)ufirst((uint32_t)v);
}
__device__ __forceinline__ bool ubool(bool b) { return ufirst(b ? 1u : 0u) != 0u; }
// v of lane l (the builtin returns a signed int: convert through uint32_t so
// that the low word of a 64-bit value is never sign-extended)
__device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t lane_value(uint64_t v, uint32_t l) {
    return ((uint64_t)lane_value((uint32_t)(v >> 32), l) << 32) | (uint64_t)lane_value((uint32_t)v, l);
}
__device__ __forceinline__ double lane_value(double v, uint32_t l) {
    return __builtin_bit_cast(double, lane_value(__builtin_bit_cast(uint64_t, v), l));
}

// Address-space views.  The pooled sums are never written while a growth
// launch runs, so uniform reads of them may go through the constant space
// (scalar loads, which do not wait on the LDS counter as flat loads do); the
// copy stack is ordinary global memory.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* as_const(const T* p) {
    return (const __attribute__((address_space(4))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Whole-record moves through those spaces, one 32-bit word at a time (the
// compiler merges them into wide loads and stores).
template <typename T>
__device__ __forceinline__ T load_const(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized record");
    T r;
    const __attribute__((address_space(4))) uint32_t* q = (const __attribute__((address_space(4))) uint32_t*)p;
    uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; ++i) d[i] = q[i];
    return r;
}
template <typename T>
__device__ __forceinline__ T load_global(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized record");
    T r;
    const __attribute__((address_space(1))) uint32_t* q = (const __attribute__((address_space(1))) uint32_t*)p;
    uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; ++i) d[i] = q[i];
    return r;
}
template <typename T>
__device__ __forceinline__ void store_global(T* p, const T& v) {
    static_assert(sizeof(T) % 4 == 0, "word-sized record");
    __attribute__((address_space(1))) uint32_t* q = (__attribute__((address_space(1))) uint32_t*)p;
    const uint32_t* d = reinterpret_cast<const uint32_t*>(&v);
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; ++i) q[i] = d[i];
}

// Direction sets of one probe window as 64-bit lane masks: direction d owns
// lanes [d*W, d*W + W); a set of directions is kept as the top bit of each
// owned field (FHI), so that "does any lane of this direction show X" is a
// field-wise nonzero test on the ballot of X.
template <int D> struct Fields;
template <> struct Fields<2> {
    static constexpr int W = 16, LW = 4;
    static constexpr uint64_t HI = 0x8000800080008000ull, LO = 0x7FFF7FFF7FFF7FFFull;
};
template <> struct Fields<3> {
    static constexpr int W = 8, LW = 3;
    static constexpr uint64_t HI = 0x0000808080808080ull, LO = 0x00007F7F7F7F7F7Full;
};

// Top bit of every field of x that has any bit set (fields never carry into
// each other: (2^(W-1) - 1) * 2 < 2^W).
template <int D>
__device__ __forceinline__ uint64_t fields_any(uint64_t x) {
    using F = Fields<D>;
    return (((x & F::LO) + F::LO) | x) & F::HI;
}

// Every lane of the fields whose top bit is set in hb.
template <int D>
__device__ __forceinline__ uint64_t fields_lanes(uint64_t hb) {
    const uint64_t x = hb >> (Fields<D>::W - 1);
    return (x << Fields<D>::W) - x;
}

// One sequence's `tours` tours against frozen pooled sums (the whole hot path
// of one walk); run by one wavefront.  Gsrc: the pooled sums to read (the
// problem's own, or an epoch's copy in a chained launch); fresh: the epoch
// starts here, so the sequence's sums and tour count start from zero instead
// of being read.  Returns the tours run, with bit 31 set if the step cap
// stopped the sequence (WALK_ABORTED).  Every value below is wave-uniform
// except where a lane index enters (scan windows, Philox counters, deletions).
// A step issues its occupancy reads first, evaluates the prune/enrich
// arithmetic while they are in flight, and only then resolves the scan.
// OBS: also record W * R^2 (squared end-to-end distance) at every arrival
// beside the weight, the numerator of the ratio estimator of eqn (5).
// LONG: walks too long for the per-length sums to share LDS with the
// occupancy table; the sums stay in the sequence's global row (read and
// written in place) and LDS holds the table, the slot ids and the stack bottom.
constexpr uint32_t WALK_ABORTED = 0x80000000u;

template <int D, bool OBS = false, bool LONG = false, bool CK = false>
__device__ __forceinline__ uint32_t walk_sequence(const ProblemDesc& P, uint32_t tours, uint32_t cap,
                                                  uint32_t s, unsigned char* lds, const SumRec* Gsrc,
                                                  bool fresh) {
    static_assert(!(OBS && CK), "observables need coordinates, which compact keys do not keep");
    using L_ = typename LatOf<D, CK>::T;
    using Key = typename L_::Key;
    using F = Fields<D>;
    constexpr int W = F::W;                    // probe positions per direction per window
    constexpr uint32_t FIELD = (1u << W) - 1u;

    // LDS: the occupancy table, the slot id of every site of the walk and the
    // sequence's own per-length sums (moved in at the start of the sequence's
    // tours and back out at their end)
    Key* table = reinterpret_cast<Key*>(lds);
    uint16_t* sid = reinterpret_cast<uint16_t*>(lds + sizeof(Key) * P.slots);
    const uint32_t row_lds = LONG ? 0u : P.row * (uint32_t)sizeof(SumRec);
    SumRec* Ls = LONG ? P.L + (size_t)s * P.row : reinterpret_cast<SumRec*>(lds + P.lds_team_bytes);
    // (observables) the sequence's per-length sums of W * R^2, after its sums
    SumRec* LRs = LONG ? P.LR + (size_t)s * P.row
                       : reinterpret_cast<SumRec*>(lds + P.lds_team_bytes + row_lds);
    // record access: LDS, or the global row of a long walk
    auto rec_ld = [&](const SumRec* p) -> SumRec {
        if constexpr (LONG) return load_global(p);
        else return *p;
    };
    auto rec_st = [&](SumRec* p, const SumRec& v) {
        if constexpr (LONG) store_global(p, v);
        else *p = v;
    };
    const int lane = (int)threadIdx.x;
    // S slots, a power of two or 1.5 times one: the home slot of a key is the
    // high word of hash * S (for S = 2^b the top b bits of the hash), and a
    // probe position past the end wraps by one subtraction (min(x, x - S) on
    // unsigned values: positions stay below 2S)
    const uint32_t S = P.slots;
    auto wrap = [S](uint32_t x) { return __builtin_elementwise_min(x, x - S); };

    // probe-lane role: direction-major, W lanes per direction (lanes past the
    // 2d directions read a slot that no mask ever selects)
    const int pdir = lane / W;
    const int poff = lane % W;
    // The walk's end is carried as its packed key; a neighbour's key is the
    // end's key moved by a per-direction offset (L_::next).  Direction 2i
    // steps +1 along axis i, direction 2i+1 steps -1; lanes past the 2d
    // directions get offset 0 (the end itself) and are never selected.
    const Key pdelta = L_::delta(pdir);
    // A zero the compiler cannot see through.  Indexing the per-length records
    // with it keeps the weight arithmetic in vector registers (the walk's
    // control state stays scalar) and lets the record read overlap the step
    // instead of being waited for on the spot to move it to scalar registers.
    uint32_t vz;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vz));

    const uint32_t n_max = P.n_max;
    const uint32_t row = P.row;
    const bool shared_mode = (P.mode == MODE_SHARED);
    const uint32_t control_mode = (P.mode != MODE_ROSENBLUTH) ? 1u : 0u;
    const double pool = shared_mode ? (double)P.N : 1.0;
    const uint64_t pool_u = shared_mode ? (uint64_t)P.N : 1ull;

    // the empty table with the origin in it, slot id of site 0
    for (uint32_t i = (uint32_t)lane; i < S; i += 64) table[i] = (Key)0;
    wave_fence();
    const Key origin_key = L_::origin();
    const uint32_t origin_slot = __umulhi(L_::hash(origin_key), S);
    if (lane == 0) {
        table[origin_slot] = origin_key;
        sid[0] = (uint16_t)origin_slot;
    }
    wave_fence();

    // the copy stack of sequence s
    StackEntry* stk = P.stack + (size_t)s * n_max;
    uint64_t MGs = shared_mode ? P.MG[0] : 0ull;

    const size_t rb0 = (size_t)s * row;
    SumRec* __restrict__ Lrow = P.L + rb0;
    const SumRec* Grow = shared_mode ? Gsrc : Gsrc + rb0;   // read with load_const
    if (!shared_mode) MGs = ufirst64(P.MG[s]);
    const uint64_t t0 = ufirst64(P.t[s]);
    uint32_t tlo = (uint32_t)t0;               // tour index: its low word keys the random numbers
    uint32_t m = fresh ? 0u : ufirst(P.m[s]);
    if constexpr (!LONG) {
        if (fresh) {
            const SumRec z = {0.0, 0, 0u};
            for (uint32_t i = (uint32_t)lane; i <= n_max; i += 64u) Ls[i] = z;
        } else {
            for (uint32_t i = (uint32_t)lane; i <= n_max; i += 64u) Ls[i] = load_global(Lrow + i);
        }
        if constexpr (OBS) {
            for (uint32_t i = (uint32_t)lane; i <= n_max; i += 64u) LRs[i] = load_global(P.LR + rb0 + i);
        }
    } else if (fresh) {
        // the sums live in the global row: an epoch that starts here clears it
        const SumRec z = {0.0, 0, 0u};
        for (uint32_t i = (uint32_t)lane; i <= n_max; i += 64u) store_global(Lrow + i, z);
        if constexpr (OBS) {
            for (uint32_t i = (uint32_t)lane; i <= n_max; i += 64u) store_global(P.LR + rb0 + i, z);
        }
    }
    wave_fence();
    SumRec rec0 = rec_ld(Ls);
    // counters of this call, added to the sequence's totals at its end: the
    // step count (scalar, it drives the cap) and one counter per lane of `cv`
    // (lane i accumulates statistics word i)
    uint32_t c_steps = 0, c_tours = 0, c_maxd = 0;
    const uint32_t capv = cap ? cap : 0xFFFFFFFFu;   // step cap of this call (0: none)
    uint64_t c_events = 0;                     // events: the sum over tours of k
    uint64_t cv = 0;
    uint32_t digest = (uint32_t)ufirst64(P.stats[(size_t)s * STATS_WORDS + ST_DIGEST]);
    bool abort = false;
    // the registers of the copy stack (see the tour loop)
    uint32_t cs_n = 0u, cs_rem = 0u;
    int32_t cs_e = 0;
    double cs_m = 0.0;
    Key cs_key = (Key)0;

    for (uint32_t tour = 0; tour < tours && !abort; ++tour) {
        // ---- a pass through the empty walk (eqn (4), M) ----
        const uint32_t tt = tlo;
        tlo += 1u;
        m += 1;
        c_tours += 1;
        XF w = {0.5, 1};                       // W_0 = 1
        {
            const XF r0 = xf_add(xf_of(rec0), w);
            rec0.m = r0.m;
            rec0.e = r0.e;
            rec0.h += 1u;
        }
        // events of this tour; fewer than 2^32 because the step cap is at most
        // 2^31 and every event either grows the walk or prunes a grown copy
        // (kb starts 64 below k, so the first event computes a block)
        uint32_t k = 0, kb = (uint32_t)-64;
        uint4 rb = make_uint4(0, 0, 0, 0);
        double ul = 0.0;                       // this lane's block as a 53-bit uniform
        uint32_t n = 0;
        Key ekey = origin_key;                 // the walk's end
        uint32_t control = 0u;                 // a decision is due at this length
        // pending copies: sp entries, the one at position p in lane p mod 64
        // of the cs_* registers for p >= lo, in global memory for p < lo (at
        // most 64 in registers; the most recent ones, which are resumed first)
        uint32_t sp = 0, lo = 0;
        XF Lc = {0.0, 0};
        SumRec Gpre = load_const(Grow);        // pooled sum of the current length
        // tours seen by the running average of eqn (6) (reading of Algorithm 2),
        // converted once per tour and kept in registers
        double seen = (double)(MGs + pool_u * (uint64_t)m);
        asm volatile("" : "+v"(seen));

        for (;;) {
            bool bt = false;
            // ---- the random block this step's event would draw (64 per pass) ----
            if (k - kb >= 64u) {
                kb = k;
                rb = philox10(make_uint4(kb + (uint32_t)lane, 0u, tt, s), P.key0, P.key1);
                // u of each lane's block, formed once per 64 events (exact:
                // integers below 2^53 and power-of-two scalings)
                ul = ((double)(rb.y >> 5) * 67108864.0 + (double)(rb.z >> 6)) * (1.0 / 9007199254740992.0);
            }
            const uint32_t li = k - kb;
            const uint32_t B0 = __builtin_amdgcn_readlane(rb.x, li);
            // pooled sums: this length's (loaded a step ago) and the next one's,
            // which the following step uses if this one grows the walk (a step
            // never starts at n_max, so n + 1 is inside the row)
            const XF Gc = xf_of(Gpre);
            const SumRec Gnx = load_const(Grow + (n + 1u));

            // ---- occupancy reads of the first window, and the next length's record ----
            // In a linear-probing run the key, if present, lies before the first
            // empty slot, so a direction is occupied iff a window shows the key
            // and free iff it shows an empty slot and no key.
            const Key nk = L_::next(ekey, pdelta);
            const uint32_t home = __umulhi(L_::hash(nk), S);
            uint32_t slot = wrap(home + (uint32_t)poff);
            Key v = table[slot];
            const SumRec nxt = rec_ld(Ls + (n + 1 + vz));
            SumRec nxr = {0.0, 0, 0u};
            if constexpr (OBS) nxr = rec_ld(LRs + (n + 1 + vz));
            __builtin_amdgcn_sched_barrier(0);

            // ---- decision arithmetic while the reads are in flight ----
            // eqn (6): r = W / [W_n], [W_n] = sum / seen (own epoch data weighted
            // N in Algorithm 2), evaluated as (W * seen) / sum; only when a
            // decision is due at this length (not after a resume or at n = 0)
            // (computed on every step and kept only when a decision is due, so
            // that the scan's first window resolves in the same block and its
            // scalar work can fill the waits of this chain)
            const XF sum = xf_add_nz(Gc, xf_mul_nz(Lc, pool));
            uint32_t ub, fi;
            {
                const double r = xf_ratio_nz(xf_mul_nz(w, seen), sum);
                const double u = lane_value(ul, li);
                const double f = floor(r);
                // bit 1: keep floor(r) copies (r integral, or u below
                // ceil(r) - r); bit 3: a walk with r < 1 survives
                ub = ufirst(((r == f || u < (f + 1.0) - r) ? 2u : 0u) | (u < r ? 8u : 0u));
                // floor(r) as an integer: r > 0, and r <= seen / N < 2^32 because
                // the sum includes N times the walk's own weight (the clamp
                // only keeps the conversion defined); r >= 1 iff fi >= 1.
                // (Converted in vector registers, then read once.)
                uint32_t fv = (uint32_t)__builtin_fmin(f, 4294967295.0);
                fi = ufirst(fv);
            }

            // ---- resolve the scan: usually the first window settles every direction ----
            uint64_t freem;                    // directions resolved free
            uint64_t insm;                     // per direction: empty lanes of the window that resolved it
            uint32_t myslot = slot;            // this lane's slot in that window
            {
                const uint64_t hd = fields_any<D>(__ballot(v == nk));
                const uint64_t empm = __ballot(v == (Key)0);
                const uint64_t ed = fields_any<D>(empm);
                freem = ed & ~hd;
                insm = empm;                   // (only fields of free directions are read)
                uint64_t pending = F::HI & ~(hd | ed);
                // scheduling groups for this block (twenty vector instructions,
                // then scalar and vector ones alternating one to two), which
                // issue a step's decision and window resolution faster than the
                // compiler's own order does
                __builtin_amdgcn_sched_group_barrier(0x002, 20, 0);
#pragma unroll
                for (int g = 0; g < 16; ++g) {
                    __builtin_amdgcn_sched_group_barrier(0x004, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
                }
                uint32_t base = (uint32_t)poff;
                while (pending != 0u) {
                    // a run longer than the window: read the next W positions
                    base += W;
                    slot = wrap(home + base);
                    v = table[slot];
                    const uint64_t act = fields_lanes<D>(pending);
                    const uint64_t hd2 = fields_any<D>(__ballot(v == nk) & act);
                    const uint64_t emp2 = __ballot(v == (Key)0) & act;
                    const uint64_t ed2 = fields_any<D>(emp2);
                    const uint64_t fr = ed2 & ~hd2;
                    freem |= fr;
                    pending &= ~(hd2 | ed2);
                    const uint64_t frl = fields_lanes<D>(fr);
                    insm = (insm & ~frl) | (emp2 & frl);
                    if ((frl >> lane) & 1u) myslot = slot;
                }
            }
            // (a 32-bit count, so that its conversion to FP64 is one instruction)
            uint32_t a = (uint32_t)__popcll(freem);
            asm volatile("" : "+s"(a));
            if (a == 0u) {
                cv += (lane == ST_TRAPS) ? 1ull : 0ull;
                bt = true;
            } else {
                k += 1;
                bool pruned = false;
                if (control) {
                    if (fi >= 1u) {
                        // r >= 1: c = floor(r) with probability ceil(r) - r, else ceil(r)
                        const uint32_t ci = (ub & 2u) ? fi : fi + 1u;
                        if (ci > 1u) {
                            w = xf_div_nz(w, (double)ci);
                            if (sp - lo == 64u) {
                                // every lane holds an entry: the oldest one moves
                                // to its place in global memory
                                if (lane == (int)(lo & 63u)) {
                                    StackEntry e;
                                    e.n = cs_n;
                                    e.remaining = cs_rem;
                                    e.e = cs_e;
                                    e.pad0 = 0u;
                                    e.m = cs_m;
                                    e.key = (uint64_t)cs_key;
                                    store_global(stk + lo, e);
                                }
                                lo += 1u;
                            }
                            // the new entry: ci - 1 copies still to resume at (n, W / ci)
                            const bool mine = lane == (int)(sp & 63u);
                            cs_n = mine ? n : cs_n;
                            cs_rem = mine ? ci - 1u : cs_rem;
                            cs_e = mine ? w.e : cs_e;
                            cs_m = mine ? w.m : cs_m;
                            cs_key = mine ? ekey : cs_key;
                            sp += 1;
                            c_maxd = (sp > c_maxd) ? sp : c_maxd;
                            cv += (lane == ST_ENRICH) ? 1ull
                                  : ((lane == ST_COPIES) ? (uint64_t)(ci - 1u) : 0ull);
                        }
                    } else if (ub & 8u) {
                        w = xf_div_nz(sum, seen);  // r < 1, survives: W / r
                    } else {
                        pruned = true;             // r < 1, pruned with probability 1 - r
                    }
                }
                if (pruned) {
                    cv += (lane == ST_PRUNES) ? 1ull : 0ull;
                    bt = true;
                } else {
                    // ---- Rosenbluth growth: the j-th free neighbour ----
                    // (the free direction whose field-top lane has exactly j
                    // free field tops below it)
                    const uint32_t j = __umulhi(B0, a);
                    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(freem >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)freem, 0u));
                    const uint64_t pick = __ballot(below == j) & freem;
                    const int dir = (__ffsll((unsigned long long)pick) - 1) >> F::LW;
                    digest = (digest ^ ((uint32_t)dir | (a << 3))) * FNV_PRIME;
                    // insertion slot: the first empty slot of the chosen direction's run
                    const uint32_t il =
                        (uint32_t)__builtin_ctz((uint32_t)(insm >> (dir * W)) & FIELD) + (uint32_t)(dir * W);
                    const uint32_t ins_slot = __builtin_amdgcn_readlane(myslot, il);
                    ekey = lane_value(nk, il);
                    // W *= a_+, eqn (2).  No range check is needed here: |e|
                    // grows by at most 3 per step and falls by at most 33 per
                    // decision, so it stays below 2^21 for every n_max allowed.
                    w = xf_mul_nz(w, (double)a);
                    n += 1;
                    c_steps += 1;
                    Gpre = Gnx;
                    // (moved to vector registers here, before the LDS writes below,
                    // so that waiting for its scalar load never waits for them)
                    asm volatile("" : "+v"(Gpre.m), "+v"(Gpre.e));
                    // ---- arrival: record into the running sums, eqn (4) ----
                    // (formed before the table insert, so that waiting for the
                    // record read never waits for the insert's LDS writes too)
                    const XF Lnew = xf_add_nz(xf_of(nxt), w);
                    SumRec nr;
                    nr.m = Lnew.m;
                    nr.e = Lnew.e;
                    nr.h = nxt.h + 1u;
                    if (lane == 0) {
                        table[ins_slot] = ekey;
                        sid[n] = (uint16_t)ins_slot;
                        rec_st(Ls + n, nr);
                    }
                    Lc = Lnew;
                    if constexpr (OBS) {
                        // R^2 of the new end, exact in FP64 (|coordinates| < 2^15)
                        int x, y, z;
                        L_::unpack(ekey, x, y, z);
                        const double r2 = (double)x * (double)x + (double)y * (double)y +
                                          (double)z * (double)z;
                        const XF R = xf_add_nz(xf_of(nxr), xf_mul_nz(w, r2));
                        SumRec rr;
                        rr.m = R.m;
                        rr.e = R.e;
                        rr.h = 0u;
                        if (lane == 0) rec_st(LRs + n, rr);
                    }
                    if (c_steps >= capv) {
                        abort = true;
                        break;
                    }
                    if (n == n_max) bt = true;
                    else control = control_mode;
                }
            }
            if (bt) {
                // ---- resume the most recent pending copy, or end the tour ----
                if (sp == 0u) break;
                if (sp == lo) {
                    // no pending entry in registers: bring back the most recent
                    // ones (up to 64) from global memory
                    const uint32_t base = sp > 64u ? sp - 64u : 0u;
                    const uint32_t q = base + (((uint32_t)lane - base) & 63u);
                    if (q < sp) {
                        const StackEntry e = load_global(stk + q);
                        cs_n = e.n;
                        cs_rem = e.remaining;
                        cs_e = e.e;
                        cs_m = e.m;
                        cs_key = (Key)e.key;
                    }
                    lo = base;
                }
                const uint32_t tl = (sp - 1u) & 63u;
                const uint32_t rn = lane_value(cs_n, tl);
                const uint32_t rem = lane_value(cs_rem, tl);
                w = XF{lane_value(cs_m, tl), (int32_t)lane_value((uint32_t)cs_e, tl)};
                ekey = (Key)lane_value(cs_key, tl);
                if (rem == 1u) sp -= 1u;       // its last copy: the entry is done
                else cs_rem -= (lane == (int)tl) ? 1u : 0u;
                // LIFO deletion of sites rn+1..n restores the table exactly
                for (uint32_t i = rn + 1u + (uint32_t)lane; i <= n; i += 64u) table[sid[i]] = (Key)0;
                n = rn;
                control = 0u;
                wave_fence();
            }
        }
        // end of the tour (or abort): back to the empty walk
        c_events += k;
        for (uint32_t i = 1u + (uint32_t)lane; i <= n; i += 64u) table[sid[i]] = (Key)0;
        wave_fence();
    }
    cv += (lane == ST_EVENTS) ? c_events : 0ull;
    if (lane == 0) rec_st(Ls, rec0);
    wave_fence();
    if constexpr (!LONG) {
        for (uint32_t i = (uint32_t)lane; i <= n_max; i += 64u) store_global(Lrow + i, Ls[i]);
        if constexpr (OBS) {
            for (uint32_t i = (uint32_t)lane; i <= n_max; i += 64u) store_global(P.LR + rb0 + i, LRs[i]);
        }
    }
    if (lane == 0) {
        if (abort) atomicOr(&P.ctrl[CTRL_ERR], ERR_CAP);
        uint64_t* sr = P.stats + (size_t)s * STATS_WORDS;
        P.t[s] = t0 + c_tours;
        P.m[s] = m;
        sr[ST_STEPS] += c_steps;
        sr[ST_TOURS] += c_tours;
        if (c_maxd > sr[ST_MAXDEPTH]) sr[ST_MAXDEPTH] = c_maxd;
        sr[ST_DIGEST] = digest;
        if (abort) sr[ST_CAPPED] = 1;
    }
    if (lane == ST_EVENTS || lane == ST_ENRICH || lane == ST_COPIES || lane == ST_PRUNES ||
        lane == ST_TRAPS)
        P.stats[(size_t)s * STATS_WORDS + lane] += cv;
    return c_tours | (abort ? WALK_ABORTED : 0u);
}

// Persistent launch over (problem, sequence) items of one or many problems:
// each wavefront takes the next item from a device queue until none is left.
// A problem alone is a batch of one, so a problem's bits do not depend on what
// else shares the launch.
template <bool OBS, bool LONG>
__device__ __forceinline__ void batch_body(const BatchArgs& B) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = (int)threadIdx.x;
    for (;;) {
        uint32_t got = 0u;
        if (lane == 0) got = atomicAdd(B.queue, 1u);
        const uint32_t item = ufirst(__shfl(got, 0, 64));
        if (item >= B.total_items) break;
        // the problem owning the item: entries are sorted by their first item
        LaunchEntry E = B.single;
        if (B.count > 1) {
            uint32_t lo = 0, hi = B.count - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (B.entries[mid].first_item <= item) lo = mid;
                else hi = mid - 1;
            }
            E = B.entries[lo];
        }
        // the descriptor is read through the constant space: a flat load would
        // make every field (and so the whole walk's control flow) non-uniform
        const ProblemDesc P = load_const(E.desc);
        const uint32_t s = item - E.first_item;
        if (P.dim == 2) walk_sequence<2, OBS, LONG>(P, E.tours, E.step_cap, s, lds, P.G, false);
        else if (!OBS && P.ckey) walk_sequence<3, false, LONG, true>(P, E.tours, E.step_cap, s, lds, P.G, false);
        else walk_sequence<3, OBS, LONG>(P, E.tours, E.step_cap, s, lds, P.G, false);
    }
}

__global__ void __launch_bounds__(64) batch_kernel(BatchArgs B) { batch_body<false, false>(B); }

// The same for one problem whose walks also record W * R^2, whose walks are
// long (sums in global memory), or both.
__global__ void __launch_bounds__(64) batch_obs_kernel(BatchArgs B) { batch_body<true, false>(B); }
__global__ void __launch_bounds__(64) batch_long_kernel(BatchArgs B) { batch_body<false, true>(B); }
__global__ void __launch_bounds__(64) batch_long_obs_kernel(BatchArgs B) { batch_body<true, true>(B); }

// ---------------------------------------------------------------------------
// Device-side epoch chaining.  Every problem runs its whole epoch schedule in
// one persistent launch: a wave claims (problem, epoch, sequence) items, runs
// the sequence's tours of that epoch, and then takes its sequence up the
// problem's merge tree -- the aligned pairwise tree over sequences, padded
// with zeros to p2 leaves -- as far as it is the second of two children to
// arrive, adding its partner's partial row into the left child's row.  The
// wave that completes the root adds the tree into the pooled sums (into a
// fresh per-epoch copy, so that scalar loads of later epochs never meet a
// line cached before it was written), adds the epoch's tours to M and
// publishes the next epoch.  The result is the same as run + merge per epoch.
// ---------------------------------------------------------------------------
constexpr uint64_t JOB_IDLE_TICKS = 100000000ull * 120ull;   // 120 s at the 100 MHz clock

__device__ __forceinline__ uint32_t job_finished(const JobArgs& A) {
    uint32_t done = 0;
    for (uint32_t c = 0; c <= A.cls; ++c)
        done += __hip_atomic_load(&A.counters[JOB_FINISHED0 + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return done;
}

// Lane 0 tries to claim the next sequence of problem pi's open epoch.
__device__ __forceinline__ bool job_claim(const JobArgs& A, uint32_t pi, uint32_t epochs, uint32_t N,
                                          bool closed, uint32_t& e, uint32_t& s) {
    unsigned long long w = __hip_atomic_load(&A.state[pi].word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int attempt = 0; attempt < 8; ++attempt) {
        const uint32_t ee = (uint32_t)(w >> 32), cc = (uint32_t)w;
        if (ee >= epochs || cc >= N || (closed && cc == 0u && ee > 0u)) return false;
        if (__hip_atomic_compare_exchange_strong(&A.state[pi].word, &w, w + 1ull, __ATOMIC_ACQUIRE,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            e = ee;
            s = cc;
            return true;
        }
    }
    return false;
}

// The sequence's part of its epoch's merge, after its tours: sample counts,
// tour count, and the climb up the merge tree.
__device__ void job_merge(const JobArgs& A, const JobProblem& J, const ProblemDesc& P, uint32_t pi,
                          uint32_t e, uint32_t s, uint32_t tours_run, unsigned char* lds) {
    const int lane = (int)threadIdx.x;
    const uint32_t row = P.row, n1 = P.n_max + 1u;
    // the sequence's sums of this epoch: in LDS, or (long walks) its global row,
    // written by this same wave
    const SumRec* Ls = J.lng ? P.L + (size_t)s * row : reinterpret_cast<const SumRec*>(lds + P.lds_team_bytes);
    for (uint32_t n = (uint32_t)lane; n < n1; n += 64u)
        __hip_atomic_fetch_add(&P.HG[n], (uint64_t)Ls[n].h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane == 0) {
        __hip_atomic_fetch_add(&A.state[pi].msum, tours_run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.m[s] = 0u;
        if (J.stage != nullptr) {
            // what the group sums of the stop rule need, before the tree overwrites the row
            store_global(J.stage + s, Ls[P.n_max]);
            J.stage_m[s] = tours_run;
        }
    }
    uint32_t l = 0, i = s;
    for (;;) {
        if (l == J.levels) break;                         // at the root
        if (((i ^ 1u) << l) < J.N) {
            // the partner subtree has leaves: the second of the two goes on
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            uint32_t old = 0u;
            if (lane == 0)
                old = __hip_atomic_fetch_add(&J.flags[(J.p2 >> (l + 1u)) + (i >> 1)], 1u, __ATOMIC_ACQ_REL,
                                             __HIP_MEMORY_SCOPE_AGENT);
            old = ufirst(__shfl(old, 0, 64));
            if (old == 0u) return;                        // the partner will continue
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane == 0) J.flags[(J.p2 >> (l + 1u)) + (i >> 1)] = 0u;
            SumRec* left = P.L + (size_t)((i & ~1u) << l) * row;
            const SumRec* right = P.L + (size_t)((i | 1u) << l) * row;
            for (uint32_t n = (uint32_t)lane; n < n1; n += 64u) {
                const SumRec a = load_global(left + n);
                const SumRec b = load_global(right + n);
                const XF v = xf_add(xf_of(a), xf_of(b));
                SumRec r;
                r.m = v.m;
                r.e = v.e;
                r.h = 0u;
                store_global(left + n, r);
            }
        }
        // (no partner: the padded subtree adds +0, the node is this subtree)
        l += 1u;
        i >>= 1;
    }
    // root: pooled sums of the next epoch, then M, then publish
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const SumRec* Gprev = (e == 0u) ? P.G : J.gver + (size_t)(e - 1u) * (row + JOB_GAP);
    SumRec* Gnext = J.gver + (size_t)e * (row + JOB_GAP);
    SumRec* Gctx = const_cast<SumRec*>(P.G);
    for (uint32_t n = (uint32_t)lane; n < n1; n += 64u) {
        const SumRec a = load_global(Gprev + n);
        const SumRec b = load_global(P.L + n);            // the root's row is leaf 0's
        const XF v = xf_add(xf_of(a), xf_of(b));
        SumRec r;
        r.m = v.m;
        r.e = v.e;
        r.h = 0u;
        store_global(Gnext + n, r);
        store_global(Gctx + n, r);
    }
    // the stop rule's group sums: lane k < 16 folds group k (sequences k, k + 16,
    // ... in order) into the context's running group sum and tour count
    double rel = __builtin_inf();
    if (J.stage != nullptr) {
        double gm = 0.0;
        int ge = 0;
        uint64_t gt = 0;
        if ((uint32_t)lane < GROUPS) {
            XF acc = {0.0, 0};
            uint64_t t = 0;
            for (uint32_t q = (uint32_t)lane; q < J.N; q += GROUPS) {
                acc = xf_add(acc, xf_of(load_global(J.stage + q)));
                t += J.stage_m[q];
            }
            const XF g = xf_add(xf_of(load_global(J.gsum + lane)), acc);
            uint64_t* gtours = reinterpret_cast<uint64_t*>(J.gsum + GROUPS);
            gt = gtours[lane] + t;
            SumRec r;
            r.m = g.m;
            r.e = g.e;
            r.h = 0u;
            store_global(J.gsum + lane, r);
            gtours[lane] = gt;
            gm = g.m;
            ge = g.e;
        }
        // the same fixed sequence of operations as the host's group_rel_err
        bool defined = true;
        int e_top = -2147483647 - 1;
        for (uint32_t k = 0; k < GROUPS; ++k) {
            const double mk = __hiloint2double((int)lane_value((uint32_t)__double2hiint(gm), k),
                                               (int)lane_value((uint32_t)__double2loint(gm), k));
            const int ek = (int)lane_value((uint32_t)ge, k);
            const uint64_t tk = lane_value(gt, k);
            if (tk == 0 || mk == 0.0) defined = false;
            else if (ek > e_top) e_top = ek;
        }
        if (defined) {
            double g[GROUPS];
            double total = 0.0;
            for (uint32_t k = 0; k < GROUPS; ++k) {
                const double mk = __hiloint2double((int)lane_value((uint32_t)__double2hiint(gm), k),
                                                   (int)lane_value((uint32_t)__double2loint(gm), k));
                const int ek = (int)lane_value((uint32_t)ge, k);
                const uint64_t tk = lane_value(gt, k);
                g[k] = ldexp(mk / (double)tk, ek - e_top);
                total += g[k];
            }
            const double mean = total / GROUPS;
            double ss = 0.0;
            for (uint32_t k = 0; k < GROUPS; ++k) ss += (g[k] - mean) * (g[k] - mean);
            rel = __builtin_sqrt(ss / (GROUPS - 1)) / (4.0 * mean);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) {
        const uint32_t msum = __hip_atomic_exchange(&A.state[pi].msum, 0u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        uint64_t* MG = const_cast<uint64_t*>(P.MG);
        const uint64_t M = MG[0] + msum;
        MG[0] = M;
        // a problem one of whose sequences hit its step cap stops after this
        // epoch (its context reports the overflow); the others run on
        const bool failed =
            __hip_atomic_load(&A.state[pi].failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        uint32_t stop = 0u;
        if (failed) stop = STOP_FAILED;
        else if (J.stage != nullptr && J.target > 0.0 && rel <= J.target) stop = STOP_TARGET;
        else if (J.cap != 0u && M >= J.cap) stop = STOP_CAP;
        if (failed) __hip_atomic_fetch_add(&A.counters[JOB_FAILED], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (J.result != nullptr) {
            J.result[0] = e + 1u;
            J.result[1] = stop;
            J.result[2] = (uint32_t)__double2loint(rel);
            J.result[3] = (uint32_t)__double2hiint(rel);
        }
        const bool last = stop != 0u || e + 1u == J.epochs;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&A.state[pi].word, (unsigned long long)(last ? J.epochs : e + 1u) << 32,
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (last)
            __hip_atomic_fetch_add(&A.counters[JOB_FINISHED0 + J.cls], 1u, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// (at most 128 VGPRs: four waves per SIMD; the register pressure this adds
// costs two spills in a chained item's merge part, none in the step loop)
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) job_kernel(JobArgs A) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = (int)threadIdx.x;
    uint64_t idle_since = __builtin_amdgcn_s_memrealtime();
    uint32_t seen_progress = 0u;
    // the slice's clock starts with the first wave to look at it
    unsigned long long* clock0 = reinterpret_cast<unsigned long long*>(A.counters + JOB_CLOCK);
    uint64_t start = 0;
    if (lane == 0) {
        unsigned long long zero = 0ull;
        const unsigned long long now0 = __builtin_amdgcn_s_memrealtime();
        __hip_atomic_compare_exchange_strong(clock0, &zero, now0, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        start = __hip_atomic_load(clock0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    start = lane_value(start, 0u);
    for (;;) {
        // past the slice's end, no epoch after a problem's first starts (the
        // started ones are finished)
        const bool closed = A.slice_ticks != 0u && __builtin_amdgcn_s_memrealtime() - start >= A.slice_ticks;
        // ---- claim: the first problem (in priority order) with an open item ----
        bool got = false;
        uint32_t pi = 0u, e = 0u, s = 0u;
        for (uint32_t b = A.start; b < A.count && !got; b += 64u) {
            const uint32_t idx = b + (uint32_t)lane;
            uint32_t mine = 0u;
            bool open = false;
            if (idx < A.count) {
                mine = A.order[idx];
                const JobProblem& J = A.probs[mine];
                const unsigned long long w =
                    __hip_atomic_load(&A.state[mine].word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // (a launch always runs each problem's first epoch, so every
                // call makes progress however short its slice)
                open = (uint32_t)(w >> 32) < J.epochs && (uint32_t)w < J.N &&
                       (!closed || (uint32_t)w > 0u || (uint32_t)(w >> 32) == 0u);
            }
            uint64_t cand = __ballot(open);
            while (cand != 0u && !got) {
                const uint32_t f = (uint32_t)__ffsll((unsigned long long)cand) - 1u;
                cand &= cand - 1u;
                const uint32_t p = lane_value(mine, f);
                uint32_t ok = 0u, ce = 0u, cs = 0u;
                if (lane == 0) {
                    const JobProblem& J = A.probs[p];
                    ok = job_claim(A, p, J.epochs, J.N, closed, ce, cs) ? 1u : 0u;
                }
                ok = ufirst(__shfl(ok, 0, 64));
                if (ok) {
                    got = true;
                    pi = p;
                    e = ufirst(__shfl(ce, 0, 64));
                    s = ufirst(__shfl(cs, 0, 64));
                }
            }
        }
        if (!got) {
            // past the slice's end nothing new becomes claimable (items are only
            // used up), so a wave that finds nothing may leave
            if (closed) break;
            if (job_finished(A) >= A.need) break;
            const uint32_t prog =
                __hip_atomic_load(&A.counters[JOB_PROGRESS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (prog != seen_progress) {
                seen_progress = prog;
                idle_since = now;
            } else if (now - idle_since > JOB_IDLE_TICKS) {
                // backstop: leave the rest to others (counted, pperm_job_report)
                if (lane == 0)
                    __hip_atomic_fetch_add(&A.counters[JOB_BACKSTOP], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(127);
            continue;
        }
        // ---- the item: the sequence's tours of this epoch, then its merge part ----
        const JobProblem J = load_const(A.probs + pi);
        const ProblemDesc P = load_const(J.desc);
        const uint32_t tours = J.sched[e];
        // the job ends with its longest chain of epochs: its waves issue first
        if (J.prio == 3u) __builtin_amdgcn_s_setprio(3);
        else if (J.prio == 2u) __builtin_amdgcn_s_setprio(2);
        else if (J.prio == 1u) __builtin_amdgcn_s_setprio(1);
        // the context's step cap, or the watchdog default of pperm_run_tours
        uint64_t cap64 = P.step_cap ? (uint64_t)P.step_cap : 4096ull * tours * (P.n_max + 1ull);
        const uint32_t cap = cap64 > (1ull << 31) ? (1u << 31) : (uint32_t)cap64;
        const SumRec* Gsrc = (e == 0u) ? P.G : J.gver + (size_t)(e - 1u) * (P.row + JOB_GAP);
        uint32_t rv;
        if (J.lng)
            rv = (P.dim == 2) ? walk_sequence<2, false, true>(P, tours, cap, s, lds, Gsrc, true)
                 : P.ckey     ? walk_sequence<3, false, true, true>(P, tours, cap, s, lds, Gsrc, true)
                              : walk_sequence<3, false, true>(P, tours, cap, s, lds, Gsrc, true);
        else
            rv = (P.dim == 2) ? walk_sequence<2>(P, tours, cap, s, lds, Gsrc, true)
                 : P.ckey     ? walk_sequence<3, false, false, true>(P, tours, cap, s, lds, Gsrc, true)
                              : walk_sequence<3>(P, tours, cap, s, lds, Gsrc, true);
        if ((rv & WALK_ABORTED) && lane == 0)
            __hip_atomic_fetch_or(&A.state[pi].failed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        job_merge(A, J, P, pi, e, s, rv & ~WALK_ABORTED, lds);
        __builtin_amdgcn_s_setprio(0);
        if (lane == 0)
            __hip_atomic_fetch_add(&A.counters[JOB_PROGRESS], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        idle_since = __builtin_amdgcn_s_memrealtime();
    }
}

// After a whole-schedule launch: every problem must have merged all of its
// epochs, or have stopped on a step cap (reported through its context
// already).  Anything else -- the launch ended early -- is flagged on the
// problem's context and counted.
__global__ void __launch_bounds__(256) job_check_kernel(JobArgs A) {
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < A.count; i += gridDim.x * 256u) {
        const JobProblem& J = A.probs[A.order[i]];
        const uint32_t done = J.result[0], stop = J.result[1];
        if (done != J.epochs && stop != STOP_FAILED) {
            atomicOr(&J.desc->ctrl[CTRL_ERR], ERR_INCOMPLETE);
            atomicAdd(&A.counters[JOB_INCOMPLETE], 1u);
        }
    }
}

__global__ void __launch_bounds__(256) fill_zero_kernel(uint32_t* p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Merge: aligned pairwise tree over sequences.  One wave takes 64 consecutive
// rows (sequences) and a strip of 16 columns (lengths); lane i holds row i and
// the tree over the 64 lanes is a butterfly of lane shuffles (xor 1, 2, ..,
// 32): after level l every lane holds the sum of its aligned block of 2^(l+1)
// rows, added as (left block) + (right block) up to commutativity, which IEEE
// addition has.  Partial trees of aligned 64-row blocks are the tree's own
// nodes, so repeated passes give the whole tree; missing rows are +0.0.
// ---------------------------------------------------------------------------
constexpr int MERGE_COLS = 8;

__global__ void __launch_bounds__(64) merge_pass_kernel(MergeArgs A) {
    const int lane = (int)threadIdx.x;
    const uint32_t r = blockIdx.y * 64u + (uint32_t)lane;
    const uint32_t c0 = blockIdx.x * MERGE_COLS;
    XF v[MERGE_COLS];
    uint64_t h[MERGE_COLS];
    const bool rv = r < A.rows;
#pragma unroll
    for (int j = 0; j < MERGE_COLS; ++j) {
        const uint32_t c = c0 + (uint32_t)j;
        const bool ok = rv && c < A.ncols;
        const size_t idx = (size_t)r * A.row + c;
        SumRec rec = {0.0, 0, 0u};
        if (ok) rec = A.in[idx];
        v[j] = xf_of(rec);
        h[j] = ok ? (A.hin ? A.hin[idx] : (uint64_t)rec.h) : 0ull;
    }
    if (A.zero && rv) {
        const SumRec z = {0.0, 0, 0u};
#pragma unroll
        for (int j = 0; j < MERGE_COLS; ++j) {
            const uint32_t c = c0 + (uint32_t)j;
            if (c < A.ncols) A.zero[(size_t)r * A.row + c] = z;
        }
    }
    // butterfly: after step lvl every lane holds the sum of its aligned block of
    // 2*lvl rows; the extended-range sum is commutative, so both lanes of a pair
    // compute the same (left block) + (right block)
#pragma unroll
    for (int lvl = 1; lvl < 64; lvl <<= 1) {
#pragma unroll
        for (int j = 0; j < MERGE_COLS; ++j) {
            XF o;
            o.m = __shfl_xor(v[j].m, lvl, 64);
            o.e = __shfl_xor(v[j].e, lvl, 64);
            v[j] = xf_add(v[j], o);
            h[j] += __shfl_xor(h[j], lvl, 64);
        }
    }
    if (lane < MERGE_COLS) {
        // select column `lane` without dynamic register indexing
        XF vv = {0.0, 0};
        uint64_t hh = 0;
#pragma unroll
        for (int j = 0; j < MERGE_COLS; ++j) {
            if (j == lane) { vv = v[j]; hh = h[j]; }
        }
        const uint32_t c = c0 + (uint32_t)lane;
        if (c < A.ncols) {
            const size_t o = (size_t)blockIdx.y * A.row + c;
            if (A.accumulate) {
                vv = xf_add(xf_of(A.out[o]), vv);
                if (A.hout) hh += A.hout[o];
            }
            SumRec rec;
            rec.m = vv.m;
            rec.e = vv.e;
            rec.h = 0u;
            A.out[o] = rec;
            if (A.hout) A.hout[o] = hh;
        }
    }
}

__global__ void __launch_bounds__(256) merge_counts_kernel(const uint32_t* m, uint32_t N,
                                                           uint64_t* MG, uint32_t* zero_m) {
    // one block: exact integer sum of the per-sequence tour counts
    __shared__ uint64_t part[256];
    uint64_t acc = 0;
    for (uint32_t i = threadIdx.x; i < N; i += 256) acc += m[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < N; i += 256) zero_m[i] = 0u;
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) MG[0] += part[0];
}

__global__ void __launch_bounds__(256) merge_independent_kernel(SumRec* L, uint32_t* m, SumRec* G,
                                                                uint64_t* HG, uint64_t* MG,
                                                                uint32_t N, uint32_t row) {
    const size_t total = (size_t)N * row;
    const SumRec z = {0.0, 0, 0u};
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (size_t)gridDim.x * 256) {
        const SumRec l = L[i];
        const XF g = xf_add(xf_of(G[i]), xf_of(l));
        SumRec rec;
        rec.m = g.m;
        rec.e = g.e;
        rec.h = 0u;
        G[i] = rec;
        HG[i] += l.h;
        L[i] = z;
    }
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
        MG[i] += m[i];
        m[i] = 0u;
    }
}

// Group sums for the error estimate: lane k < 16 folds the records at n_max of
// sequences k, k + 16, k + 32, ... (in that order, from zero) and adds the
// result to the group's running total; tours likewise.  Runs before the merge
// that zeroes the records.
__global__ void __launch_bounds__(64) group_sums_kernel(const SumRec* L, const uint32_t* m,
                                                        uint32_t N, uint32_t row, uint32_t n_max,
                                                        SumRec* gsum, uint64_t* gtours) {
    const uint32_t k = threadIdx.x;
    if (k >= GROUPS) return;
    XF acc = {0.0, 0};
    uint64_t tours = 0;
    for (uint32_t s = k; s < N; s += GROUPS) {
        acc = xf_add(acc, xf_of(L[(size_t)s * row + n_max]));
        tours += m[s];
    }
    const XF g = xf_add(xf_of(gsum[k]), acc);
    SumRec r;
    r.m = g.m;
    r.e = g.e;
    r.h = 0u;
    gsum[k] = r;
    gtours[k] += tours;
}

__global__ void reset_ctrl_kernel(uint32_t* ctrl) {
    if (threadIdx.x == CTRL_QUEUE) ctrl[CTRL_QUEUE] = 0u;
}

__global__ void __launch_bounds__(256) init_state_kernel(uint64_t* stats, uint32_t N,
                                                         uint32_t* zero, size_t words) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (size_t)gridDim.x * 256)
        zero[i] = 0u;
    // stats rows: counters 0, digest = the FNV-1a 32 offset basis
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256)
        stats[i * STATS_WORDS + ST_DIGEST] = FNV_OFFSET;
}

template <int D, int TS>
hipError_t launch_run_t(const RunArgs& a, uint32_t wgs, uint32_t lds, hipStream_t s) {
    hipLaunchKernelGGL((run_kernel<D, TS>), dim3(wgs), dim3(64), lds, s, a);
    return hipGetLastError();
}

template <int D, int TS>
hipError_t occupancy_t(uint32_t lds, int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, run_kernel<D, TS>, 64, lds);
}

}  // namespace

hipError_t launch_reset_ctrl(uint32_t* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(reset_ctrl_kernel, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

hipError_t launch_init_state(uint64_t* stats, uint32_t N, void* zero_base, size_t zero_bytes,
                             hipStream_t s) {
    // zero everything first, then the digest seeds: same kernel, in order
    const size_t words = zero_bytes / 4;
    uint32_t blocks = (uint32_t)((words + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(init_state_kernel, dim3(blocks), dim3(256), 0, s, (uint64_t*)nullptr, 0u,
                       (uint32_t*)zero_base, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(init_state_kernel, dim3((N + 255) / 256), dim3(256), 0, s, stats, N,
                       (uint32_t*)nullptr, (size_t)0);
    return hipGetLastError();
}

#define PPERM_TS_SWITCH(D, FN, ...)                                     \
    switch (team_lanes) {                                               \
        case 4: if (D == 2) return FN<2, 4>(__VA_ARGS__); break;        \
        case 8: return FN<D, 8>(__VA_ARGS__);                           \
        case 16: return FN<D, 16>(__VA_ARGS__);                         \
        case 32: return FN<D, 32>(__VA_ARGS__);                         \
        case 64: return FN<D, 64>(__VA_ARGS__);                         \
        default: break;                                                 \
    }

hipError_t launch_batch(const BatchArgs& b, uint32_t workgroups, uint32_t lds_bytes, hipStream_t s,
                        bool observables, bool long_walk) {
    const dim3 g(workgroups), t(64);
    if (long_walk && observables) hipLaunchKernelGGL(batch_long_obs_kernel, g, t, lds_bytes, s, b);
    else if (long_walk) hipLaunchKernelGGL(batch_long_kernel, g, t, lds_bytes, s, b);
    else if (observables) hipLaunchKernelGGL(batch_obs_kernel, g, t, lds_bytes, s, b);
    else hipLaunchKernelGGL(batch_kernel, g, t, lds_bytes, s, b);
    return hipGetLastError();
}

hipError_t launch_job(const JobArgs& a, uint32_t workgroups, uint32_t lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(job_kernel, dim3(workgroups), dim3(64), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_job_check(const JobArgs& a, hipStream_t s) {
    const uint32_t blocks = (a.count + 255u) / 256u;
    hipLaunchKernelGGL(job_check_kernel, dim3(blocks ? blocks : 1u), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t job_occupancy(uint32_t lds_bytes, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, job_kernel, 64, lds_bytes);
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    uint32_t blocks = (uint32_t)((words + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, words);
    return hipGetLastError();
}

hipError_t batch_occupancy(uint32_t lds_bytes, int* blocks_per_cu, bool long_walk) {
    if (long_walk) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_long_kernel, 64, lds_bytes);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_kernel, 64, lds_bytes);
}

hipError_t launch_run(const RunArgs& a, uint32_t dim, uint32_t team_lanes, uint32_t workgroups,
                      uint32_t lds_bytes, hipStream_t s) {
    if (dim == 2) {
        PPERM_TS_SWITCH(2, launch_run_t, a, workgroups, lds_bytes, s)
    } else if (dim == 3) {
        PPERM_TS_SWITCH(3, launch_run_t, a, workgroups, lds_bytes, s)
    }
    return hipErrorInvalidValue;
}

hipError_t run_kernel_lds_ok(uint32_t dim, uint32_t team_lanes, uint32_t lds_bytes,
                             int* blocks_per_cu) {
    if (team_lanes == 64) return batch_occupancy(lds_bytes, blocks_per_cu);
    if (dim == 2) {
        PPERM_TS_SWITCH(2, occupancy_t, lds_bytes, blocks_per_cu)
    } else if (dim == 3) {
        PPERM_TS_SWITCH(3, occupancy_t, lds_bytes, blocks_per_cu)
    }
    return hipErrorInvalidValue;
}

hipError_t launch_merge_pass(const MergeArgs& a, hipStream_t s) {
    dim3 grid((a.ncols + MERGE_COLS - 1) / MERGE_COLS, (a.rows + 63) / 64);
    hipLaunchKernelGGL(merge_pass_kernel, grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_merge_counts(const uint32_t* m, uint32_t N, uint64_t* MG, uint32_t* zero_m,
                               hipStream_t s) {
    hipLaunchKernelGGL(merge_counts_kernel, dim3(1), dim3(256), 0, s, m, N, MG, zero_m);
    return hipGetLastError();
}

hipError_t launch_group_sums(const SumRec* L, const uint32_t* m, uint32_t N, uint32_t row,
                             uint32_t n_max, SumRec* gsum, uint64_t* gtours, hipStream_t s) {
    hipLaunchKernelGGL(group_sums_kernel, dim3(1), dim3(64), 0, s, L, m, N, row, n_max, gsum, gtours);
    return hipGetLastError();
}

hipError_t launch_merge_independent(SumRec* L, uint32_t* m, SumRec* G, uint64_t* HG, uint64_t* MG,
                                    uint32_t N, uint32_t row, hipStream_t s) {
    size_t total = (size_t)N * row;
    uint32_t blocks = (uint32_t)((total + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(merge_independent_kernel, dim3(blocks), dim3(256), 0, s, L, m, G, HG, MG,
                       N, row);
    return hipGetLastError();
}

}  // namespace pperm

// Scratch of the allocation-free batched launch (pperm_run_batch_noalloc): the
// queue words of its launches, then one launch entry per problem.  Each device
// the library runs on holds its own copy for the life of the process; calls on
// one device share it.
static __device__ __align__(256) unsigned char
    scratch[pperm::NOALLOC_QUEUE_BYTES + pperm::NOALLOC_MAX_PROBLEMS * sizeof(pperm::LaunchEntry)];

// The device address of `scratch` on the current device, looked up once per
// device with that device current (the host-side name of the array is not a
// device address and must never reach a kernel or a copy).
hipError_t pperm::noalloc_scratch(void** ptr, size_t* bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = sizeof(scratch);
    return hipSuccess;
}
