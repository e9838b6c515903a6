// The batched run of Sec. 2.2 (several bursts, several mini-stacks each) as
// one persistent launch.  Every (item, stage) pair is a segment of work
// units; segments are queued in dependency order (level by level, and within
// a level statistics, GLRT, coherence, linking, compression), and a
// workgroup takes the next unit from one device-wide counter.  Before the
// first unit of a segment it waits until the segments it depends on are
// complete: the item's previous stage, and for coherence the compression of
// every item whose compressed SLC it reads (the kappa halo of Fig. 1).  A
// workgroup publishes its completed units of a segment (release fence, then
// one atomic add) when it moves to another segment or finishes, and never
// waits while holding unpublished units, so units handed out earlier always
// complete: no deadlock, whatever the number of resident workgroups.  All
// counters only grow; run r waits for (r + 1) x units, so a replayed graph
// needs no reset.  Waits are bounded: past the bound the error word is set
// and the workgroup goes on, so the launch always ends.
//
// Workgroups of 512 threads: the coherence body uses all of them; the
// one-thread-per-item stages and linking run two 256-thread blocks side by
// side.
#include "batch_device.hpp"
#include "coherence_device.hpp"
#include "compress_device.hpp"
#include "glrt_device.hpp"
#include "link_device.hpp"
#include "stats_device.hpp"

namespace plk {
namespace {

constexpr int kMegaThreads = 512;

// The unit's pixel groups (four pixels per wavefront, four per block) go to
// the workgroup's wavefronts one at a time from a counter in LDS, so a
// wavefront that finishes early takes the next group: the unit then ends
// with at most one group of imbalance rather than a wavefront's whole share.
template <int R, int NJ>
__device__ __forceinline__ void mega_link(const LinkArgs& a, int64_t b0, int64_t b1, uint32_t* lds, int* next) {
    const int phys = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float2* l = reinterpret_cast<float2*>(lds) + (phys >> 2) * (link_lds_bytes<R, NJ>() / 8);
    const int groups = (int)(b1 - b0) * (kBlock / 64);
    for (;;) {
        int g = 0;
        if (lane == 0) g = atomicAdd(next, 1);
        g = __builtin_amdgcn_readfirstlane(g);
        if (g >= groups) break;
        const int64_t b = b0 + g / (kBlock / 64);
        link_body<R, NJ>(a, b, ((g % (kBlock / 64)) << 6) | lane, l, phys & 3);
    }
}

template <bool SPLIT>
__device__ __forceinline__ void mega_unit(const MegaPlan& p, const MegaSeg& S, int64_t unit, uint32_t* lds,
                                          int* next) {
    const int64_t b0 = unit * S.per_unit;
    const int64_t b1 = b0 + S.per_unit < S.blocks ? b0 + S.per_unit : S.blocks;
    const int sub = threadIdx.x / kBlock, tid = threadIdx.x % kBlock;
    switch (S.stage) {
        // the streaming stages take two blocks per 256-thread half at a time,
        // so that both blocks' loads are in flight together
        case MS_STATS_VEC:
            for (int64_t b = b0 + sub; b < b1; b += 4) {
                stats_vec_body(p.stats[S.arg], b, tid);
                if (b + 2 < b1) stats_vec_body(p.stats[S.arg], b + 2, tid);
            }
            break;
        case MS_STATS_SCALAR:
            for (int64_t b = b0 + sub; b < b1; b += 4) {
                stats_scalar_body(p.stats[S.arg], b, tid);
                if (b + 2 < b1) stats_scalar_body(p.stats[S.arg], b + 2, tid);
            }
            break;
        case MS_GLRT: {
            // each half of the workgroup a tile of its own (TX * TY <= 256
            // threads), its scale tile in its own half of the LDS; a block
            // past the item's last (odd count) loads NaN and writes nothing
            const GlrtArgs& a = p.glrt[S.arg];
            const int64_t nblk = a.gx * ((a.g.oR + a.TY - 1) / a.TY);
            double* tile = reinterpret_cast<double*>(lds) + sub * (int64_t)a.tw * a.th;
            for (int64_t b = b0; b < b1; b += 2) {
                const int64_t bb = b + sub < b1 ? b + sub : nblk;
                glrt_body(a, bb % a.gx, bb / a.gx, tile, tid, kBlock);
                __syncthreads();  // the tiles are refilled by the next blocks
            }
            break;
        }
        case MS_COH16:
        case MS_COH32: {
            const CohArgs a = p.coh[S.arg];
            for (int64_t b = b0; b < b1; ++b) {
                // the body ends with a workgroup barrier
                if (S.stage == MS_COH16)
                    coherence_body<16, SPLIT>(a, p.coh[S.arg].t.p, b % a.n_strips, b / a.n_strips, lds);
                else
                    coherence_body<32, SPLIT>(a, p.coh[S.arg].t.p, b % a.n_strips, b / a.n_strips, lds);
            }
            break;
        }
        case MS_COMPRESS: {
            // four blocks per half at a time: their plane loads are in flight
            // together (one workgroup per CU leaves few wavefronts to hide
            // the memory latency otherwise)
            const CompressArgs& a = p.comp[S.arg];
            for (int64_t b = b0 + sub; b < b1; b += 8) compress_body4(a, b, b1, tid);
            break;
        }
        default: {
            const LinkArgs& a = p.link[S.arg];
            switch (S.stage - MS_LINK) {
                case 1: case 2: case 3: mega_link<1, 12>(a, b0, b1, lds, next); break;
                case 4: mega_link<1, 16>(a, b0, b1, lds, next); break;
                case 5: mega_link<2, 20>(a, b0, b1, lds, next); break;
                case 6: mega_link<2, 24>(a, b0, b1, lds, next); break;
                case 7: mega_link<2, 28>(a, b0, b1, lds, next); break;
                default: mega_link<2, 32>(a, b0, b1, lds, next); break;
            }
        }
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(kMegaThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void batch_mega(MegaPlan p) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ long long s_unit;
    __shared__ int s_seg;
    __shared__ int s_next;  // pixel groups of a linking unit handed out so far
    const unsigned run = __hip_atomic_load(p.run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long base = (unsigned long long)run * (unsigned long long)(p.total + gridDim.x);
    int cur = -1, pend_seg = -1;  // meaningful in thread 0
    unsigned pend = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned long long u = atomicAdd(p.queue, 1ull) - base;
            int sg = -1;
            if (u < (unsigned long long)p.total) {  // last segment starting at or before u
                int lo = 0, hi = p.nseg - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (p.seg_start[mid] <= (long long)u) lo = mid;
                    else hi = mid - 1;
                }
                sg = lo;
            }
            if (pend && sg != pend_seg) {  // publish before moving on (or waiting)
                __threadfence();
                atomicAdd(p.done + pend_seg, (unsigned long long)pend);
                pend = 0;
            }
            if (sg >= 0 && sg != cur) {
                const MegaSeg& S = p.seg[sg];
                for (int d = 0; d < S.ndep; ++d) {
                    const int ds = S.dep[d];
                    const unsigned long long need = (unsigned long long)(run + 1) * (unsigned long long)p.seg[ds].units;
                    unsigned spins = 0;
                    while (__hip_atomic_load(p.done + ds, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (++spins > p.spin_limit) {
                            atomicOr(p.error, 1u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
                __threadfence();
            }
            s_unit = (long long)u;
            s_seg = sg;
            s_next = 0;
        }
        __syncthreads();
        const int sg = s_seg;
        const long long u = s_unit;
        if (sg < 0) break;
        cur = sg;
        mega_unit<SPLIT>(p, p.seg[sg], u - p.seg_start[sg], lds, &s_next);
        __syncthreads();  // the unit is done; s_unit and s_seg may be rewritten
        if (threadIdx.x == 0) {
            pend_seg = sg;
            ++pend;
        }
    }
    if (threadIdx.x == 0) {
        if (pend) {
            __threadfence();
            atomicAdd(p.done + pend_seg, (unsigned long long)pend);
        }
        __threadfence();
        // the last workgroup of this run moves the run counter on
        if (atomicAdd(p.finished, 1u) == (run + 1) * gridDim.x - 1) atomicAdd(p.run, 1u);
    }
}

}  // namespace

int mega_threads() { return kMegaThreads; }

const void* mega_fn(bool split) {
    return split ? reinterpret_cast<const void*>(batch_mega<true>) : reinterpret_cast<const void*>(batch_mega<false>);
}

size_t mega_link_lds(int N_class) {
    switch (N_class) {
        case 1: case 2: case 3: return 2 * (size_t)link_lds_bytes<1, 12>();
        case 4: return 2 * (size_t)link_lds_bytes<1, 16>();
        case 5: return 2 * (size_t)link_lds_bytes<2, 20>();
        case 6: return 2 * (size_t)link_lds_bytes<2, 24>();
        case 7: return 2 * (size_t)link_lds_bytes<2, 28>();
        default: return 2 * (size_t)link_lds_bytes<2, 32>();
    }
}

pl_status launch_mega(const MegaPlan& p, bool split, size_t lds, int64_t grid, hipStream_t s) {
    if (split) hipLaunchKernelGGL((batch_mega<true>), dim3((unsigned)grid), dim3(kMegaThreads), lds, s, p);
    else hipLaunchKernelGGL((batch_mega<false>), dim3((unsigned)grid), dim3(kMegaThreads), lds, s, p);
    return launch_ok("single-launch batched run");
}

}  // namespace plk
