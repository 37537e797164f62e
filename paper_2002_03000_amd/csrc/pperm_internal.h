// Internal interface between the host C-ABI layer and the gfx950 kernels of
// libpperm.so.  Not installed, not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef struct pperm_config pperm_config;

namespace pperm {

// Error bits a kernel may raise in ctrl[1]: the step cap stopped a sequence; a
// weight left the exponent range; a chained launch ended before every epoch
// it was given for the context had run.
enum : uint32_t { ERR_CAP = 1u, ERR_RANGE = 2u, ERR_INCOMPLETE = 4u };

// Exponents beyond this magnitude are reported as PPERM_ERANGE.
constexpr int32_t EXP_LIMIT = 1 << 30;

// Control words in the workspace.
enum : uint32_t { CTRL_QUEUE = 0, CTRL_ERR = 1, CTRL_WORDS = 16 };

// Modes (same values as the ABI).
enum : uint32_t { MODE_SHARED = 0, MODE_INDEPENDENT = 1, MODE_ROSENBLUTH = 2 };

// Longest cubic walk whose sites are keyed in 32 bits (10 bits per coordinate
// modulo 1024, see Lat3c): n_max + 1 < 1024.
constexpr uint32_t COMPACT3_MAX_N = 1022;

constexpr int STATS_WORDS = 10;
constexpr uint32_t GROUPS = 16;   // sequence groups of the error estimate (s mod 16)
enum : int { ST_STEPS = 0, ST_EVENTS, ST_ENRICH, ST_COPIES, ST_PRUNES, ST_TRAPS,
             ST_TOURS, ST_MAXDEPTH, ST_DIGEST, ST_CAPPED };

// 16-byte record of an extended-range sum: value = m * 2^e (m in [0.5, 1) or
// m = 0 and e = 0) and, for the per-sequence sums, the sample count h.
struct __attribute__((aligned(16))) SumRec {
    double m;
    int32_t e;
    uint32_t h;
};

// 32-byte pending-copy entry: the length and weight (m * 2^e) the copies
// resume from, how many are still pending, and the packed endpoint site.
struct __attribute__((aligned(16))) StackEntry {
    uint32_t n;
    uint32_t remaining;
    int32_t e;
    uint32_t pad0;
    double m;
    uint64_t key;
};

struct RunArgs {
    const SumRec* G;      // shared: [row]; independent: [N][row]
    const uint64_t* MG;   // shared: [1];   independent: [N]
    SumRec* L;            // [N][row]
    uint32_t* m;          // [N]
    uint64_t* t;          // [N]
    uint64_t* stats;      // [N][STATS_WORDS]
    StackEntry* stack;    // [stack_slots][n_max]
    uint32_t* ctrl;       // CTRL_WORDS
    uint32_t N;
    uint32_t n_max;
    uint32_t row;
    uint32_t tours;
    uint32_t mode;
    uint32_t slots_log2;
    uint32_t lds_team_bytes;
    uint32_t key0, key1;
    uint32_t step_cap;
};

// Everything the growth kernel needs to know about one problem; written once
// into the problem's workspace when its context is created.
struct ProblemDesc {
    SumRec* L;            // [N][row]
    const SumRec* G;      // shared: [row]; independent: [N][row]
    const uint64_t* MG;   // shared: [1];   independent: [N]
    uint64_t* HG;         // shared: [row]; independent: [N][row]
    uint32_t* m;          // [N]
    uint64_t* t;          // [N]
    uint64_t* stats;      // [N][STATS_WORDS]
    StackEntry* stack;    // [N][n_max]
    uint32_t* ctrl;       // CTRL_WORDS
    uint32_t dim;
    uint32_t N;
    uint32_t n_max;
    uint32_t row;
    uint32_t mode;
    uint32_t slots_log2;
    uint32_t lds_team_bytes;   // occupancy table + slot ids; the sums row follows
    uint32_t key0, key1;
    uint32_t step_cap;    // the configuration's step cap per sequence and call (0: default)
    SumRec* LR;           // [N][row] per-sequence sums of W * R^2, or nullptr
    uint32_t ckey;        // 1: cubic walks with 32-bit keys (n_max <= COMPACT3_MAX_N)
    uint32_t slots;       // occupancy-table slots of one walk (wave per walk)
};

// One problem's share of a launch: its tours, its step cap, and the index of
// its first (problem, sequence) item in the launch's queue.
struct LaunchEntry {
    const ProblemDesc* desc;
    uint32_t tours;
    uint32_t step_cap;
    uint32_t first_item;
    uint32_t pad;
};

struct BatchArgs {
    const LaunchEntry* entries;   // count > 1: sorted by first_item
    LaunchEntry single;           // count == 1
    uint32_t count;
    uint32_t total_items;
    uint32_t* queue;              // zeroed before the launch
};

struct MergeArgs {
    const SumRec* in;      // [rows][row]
    SumRec* out;           // [ceil(rows/64)][row], or G when final
    uint64_t* hout;        // [ceil(rows/64)][row], or HG when final; nullptr: no counts
    const uint64_t* hin;   // later passes: [rows][row]; first pass: nullptr (counts in `in`)
    SumRec* zero;          // input to clear after reading (first pass) or nullptr
    uint32_t rows;
    uint32_t row;
    uint32_t ncols;        // n_max + 1
    uint32_t accumulate;   // final pass: out[n] = out[n] + tree
};

// Launchers (pperm_kernels.hip).  All return the hipError_t of the launch.
hipError_t launch_reset_ctrl(uint32_t* ctrl, hipStream_t s);
hipError_t launch_init_state(uint64_t* stats, uint32_t N, void* zero_base, size_t zero_bytes,
                             hipStream_t s);
hipError_t launch_run(const RunArgs& a, uint32_t dim, uint32_t team_lanes, uint32_t workgroups,
                      uint32_t lds_bytes, hipStream_t s);
hipError_t run_kernel_lds_ok(uint32_t dim, uint32_t team_lanes, uint32_t lds_bytes,
                             int* blocks_per_cu);
hipError_t launch_merge_pass(const MergeArgs& a, hipStream_t s);
// Device-side epoch chaining (pperm_run_job): one problem's part.
struct JobProblem {
    const ProblemDesc* desc;
    const uint32_t* sched;    // tours per sequence of each epoch
    SumRec* gver;             // [epochs][row]: pooled sums after each epoch's merge
    uint32_t* flags;          // [p2] merge-tree node flags, zero between uses
    uint32_t epochs;
    uint32_t N;
    uint32_t p2;              // N rounded up to a power of two
    uint32_t levels;          // log2(p2)
    uint32_t cls;             // LDS class
    uint32_t lds;             // LDS bytes its walks need
    uint32_t prio;            // issue priority 0..3 of its waves (longest chains highest)
    uint32_t lng;             // 1: long walks, the sequences' sums live in global memory
    // stop rule (evaluated after every merge; stage == nullptr: none)
    SumRec* stage;            // [N] each sequence's record at n_max in the open epoch
    uint32_t* stage_m;        // [N] its tours in the open epoch
    SumRec* gsum;             // the context's 16 group sums, then 16 u64 group tours
    uint32_t* result;         // [4]: epochs done, stop reason (1 target, 2 cap), rel. error (2 words)
    double target;            // relative-error target, 0: none
    uint64_t cap;             // stop once the pooled tours M reach this, 0: none
};

// Per-problem scheduling word: (epoch << 32) | sequences claimed in it; the
// tours of the epoch's finished sequences; and a flag raised when one of the
// problem's sequences hit its step cap (the problem then stops after that
// epoch).
struct JobState {
    unsigned long long word;
    uint32_t msum;
    uint32_t failed;
};

// Counter words of a chained launch (at offset 0 of its workspace):
// problems finished per LDS class, items completed, problems stopped by a
// step cap, waves that left on the idle backstop, problems whose epochs did
// not all run, and the slice's start time (two words).
enum : uint32_t { JOB_FINISHED0 = 0, JOB_PROGRESS = 4, JOB_FAILED = 5, JOB_BACKSTOP = 6,
                  JOB_INCOMPLETE = 7, JOB_CLOCK = 8, JOB_COUNTER_WORDS = 16 };
// stop reasons a chained problem records: error target, tour cap, step cap
enum : uint32_t { STOP_TARGET = 1, STOP_CAP = 2, STOP_FAILED = 3 };
// records between consecutive per-epoch copies of the pooled sums (256 bytes)
constexpr uint32_t JOB_GAP = 16;

struct JobArgs {
    const JobProblem* probs;
    JobState* state;
    const uint32_t* order;    // problem indices: classes descending, longest chain first
    uint32_t* counters;       // JOB_* words
    uint32_t count;
    uint32_t start;           // first position of `order` this launch's waves may take
    uint32_t cls;             // this launch's LDS class
    uint32_t need;            // problems of classes <= cls
    uint64_t slice_ticks;     // 100 MHz ticks after which no epoch starts, 0: none
};

hipError_t launch_job(const JobArgs& a, uint32_t workgroups, uint32_t lds_bytes, hipStream_t s);
// After a whole-schedule launch: flag the context of every problem whose
// epochs did not all run (ERR_INCOMPLETE) and count them.
hipError_t launch_job_check(const JobArgs& a, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t job_occupancy(uint32_t lds_bytes, int* blocks_per_cu);

// True for a valid configuration whose walks run with their per-length sums
// in global memory (one problem per launch only).
bool config_long_walk(const pperm_config* c);

hipError_t launch_batch(const BatchArgs& b, uint32_t workgroups, uint32_t lds_bytes, hipStream_t s,
                        bool observables = false, bool long_walk = false);
hipError_t batch_occupancy(uint32_t lds_bytes, int* blocks_per_cu, bool long_walk = false);

// The file-scope scratch of the allocation-free batched launch on the current
// device: its device address (looked up once per device) and size.  Holds the
// queue words (first 256 bytes) and the launch entries.
constexpr uint32_t NOALLOC_MAX_PROBLEMS = 4096;
constexpr size_t NOALLOC_QUEUE_BYTES = 256;
hipError_t noalloc_scratch(void** ptr, size_t* bytes);
hipError_t launch_merge_counts(const uint32_t* m, uint32_t N, uint64_t* MG, uint32_t* zero_m,
                               hipStream_t s);
hipError_t launch_group_sums(const SumRec* L, const uint32_t* m, uint32_t N, uint32_t row,
                             uint32_t n_max, SumRec* gsum, uint64_t* gtours, hipStream_t s);
hipError_t launch_merge_independent(SumRec* L, uint32_t* m, SumRec* G, uint64_t* HG, uint64_t* MG,
                                    uint32_t N, uint32_t row, hipStream_t s);

}  // namespace pperm
