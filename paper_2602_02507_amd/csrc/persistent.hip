// Persistent batched solve: every phase of every field of a batch in one
// launch, over device work queues.
//
// A field's work is its phases in solve order (packing, FP16 row split,
// moment contraction, split-K sum, radial scan, coefficient step, expansion
// contraction, broadcast of merged blocks); phase h is a run of items, each
// item a group of consecutive workgroups of the phase's own kernel (several
// for the light phases, so that the cost of taking an item is spread over
// enough work), run with the same device code, so results are bitwise those
// of the per-phase launches.
//
// The host lays the items out as one queue per XCD (an accelerator complex
// die, with its own L2): whole fields, spread over the queues by their
// estimated work and ordered shortest first within a queue, so that small
// fields finish early.  A workgroup reads the id of the XCD it runs on,
// takes the next item of that XCD's queue (an atomic dispenser), waits until
// every item of the field's previous phase has completed, runs the item and
// counts it complete.  All items of a field run on one XCD, so producers and
// consumers share one L2; within the launch every intermediate is written
// once before it is read (and no CU has read it before), so a producer only
// needs its stores completed (s_waitcnt vmcnt(0)) before it counts the item,
// and no cache has to be written back or invalidated.  An item waits only on
// items dispensed before it from the same queue, which are held by running
// workgroups, so the waits always end; still, every wait is bounded: past
// spin_limit polls it sets the error word, counts the item without running
// it (so later waits end too) and the launch ends normally; the host reports
// the error after synchronising.
#define MPOLE_ITEM_LOOP 1
#include "bcast_impl.h"
#include "coef_impl.h"
#include "gemm_f64_impl.h"
#include "gemm_split_impl.h"
#include "pack_impl.h"
#include "scan_impl.h"

namespace mpole {
namespace {

constexpr int PERSIST_THREADS = 256;
constexpr int PERSIST_SCAN_MODES = PERSIST_THREADS / SCAN_CHUNKS;   // 4 modes x 64 radial chunks
static_assert(PERSIST_SCAN_MODES * SCAN_CHUNKS == PERSIST_THREADS, "scan workgroup");
static_assert(PACK_THREADS == PERSIST_THREADS && NTH == PERSIST_THREADS && NTHREADS == PERSIST_THREADS,
              "every item runs on the workgroup shape of its per-phase kernel");

// id of the XCD this workgroup runs on (hardware register XCC_ID, bits 3:0)
__device__ inline int xcc_id() { return __builtin_amdgcn_s_getreg(6164) & 15; }

template <int KIND>
constexpr int persist_lds_bytes() {
  constexpr int gemm = KIND == 0 ? F64_LDS * 8 : split_lds_slots<KIND == 0 ? kSplitBf16x3 : KIND>() * 16;
  constexpr int pack = KIND == kSplitBf16x3 ? PACK_LDS : 256;
  constexpr int scan = scan_lds<PERSIST_SCAN_MODES>() * 8;
  return gemm > pack ? (gemm > scan ? gemm : scan) : (pack > scan ? pack : scan);
}

// Item idx of queue q: (field, phase, item within the phase), or false past
// the end.  The search starts from the segment of the previous item of this
// workgroup (`seg`, updated): a queue's indices only grow.
__device__ inline bool decode(const PersistDev &Q, int q, uint32_t idx, int &seg, int &f, int &h, int &local) {
  int lo = max(Q.qseg[q], seg), hi = Q.qseg[q + 1] - 1;
  if (hi < lo) return false;
  const int4 last = Q.segs[hi];
  if (idx >= (uint32_t)(last.z + last.w)) return false;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint32_t)Q.segs[mid].z <= idx) lo = mid; else hi = mid - 1;
  }
  const int4 s = Q.segs[lo];
  seg = lo;
  f = s.x;
  h = s.y;
  local = (int)idx - s.z;
  return true;
}

// The queue descriptor and the batch descriptor (the kernel's first argument,
// at offset 0 of the kernel argument segment) are read through addresses
// made opaque in each iteration, so that their loads are not hoisted out of
// the loop: held across an item, they would crowd out the item's registers.
template <int KIND>
__global__ __launch_bounds__(PERSIST_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_persistent(
    BatchDev Bk, const PersistDev *Qp, uint32_t spin_limit) {
  __shared__ __align__(16) char lds[persist_lds_bytes<KIND>()];
  __shared__ int4 item;   // field, phase (-1: skip, -2: leave), first and end sub-item
  const int q = Qp->xcc_q[xcc_id()];
  if (q < 0) return;   // an XCD the queues do not cover (not seen when the batch was bound)
  if (Bk.stamps != nullptr && blockIdx.x == 0 && threadIdx.x == 0) Bk.stamps[Bk.nf] = wall_clock64();
  int seg = 0;   // thread 0: segment of the previous item
  for (;;) {
    if (threadIdx.x == 0) {
      const PersistDev *qd = Qp;
      __asm__ volatile("" : "+v"(qd));
      const PersistDev Q = *qd;
      int f = 0, h = 0, local = 0, s0 = 0, s1 = 0;
      if (!decode(Q, q, atomicAdd(&Q.next[q], 1u), seg, f, h, local)) {
        h = -2;
      } else {
        // the field's previous phase with items must be complete
        int hp = h - 1;
        while (hp >= 0 && Q.tot[f * PH_COUNT + hp] == 0) --hp;
        bool run = true;
        if (hp >= 0) {
          const uint32_t need = (uint32_t)Q.tot[f * PH_COUNT + hp];
          uint32_t polls = 0;
          while (atomicAdd(&Q.done[f * PH_COUNT + hp], 0u) < need) {
            if (++polls > spin_limit) {
              atomicOr(Q.err, 1u);
              run = false;   // skip the item; the batch result is undefined, the host reports it
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
        if (run) {
          const int g = Q.grp[f * PH_COUNT + h];
          s0 = local * g;
          s1 = min(s0 + g, Q.sub[f * PH_COUNT + h]);
        } else {
          // still count it, so that the later phases of the field stop waiting too
          atomicAdd(&Q.done[f * PH_COUNT + h], 1u);
          h = -1;
        }
      }
      item = int4{f, h, s0, s1};
    }
    __syncthreads();
    // workgroup-uniform: the plan descriptor below then goes to scalar registers
    const int f = __builtin_amdgcn_readfirstlane(item.x), h = __builtin_amdgcn_readfirstlane(item.y);
    const int s0 = __builtin_amdgcn_readfirstlane(item.z), s1 = __builtin_amdgcn_readfirstlane(item.w);
    if (h == -2) break;
    if (h >= 0) {
      for (int s = s0; s < s1; ++s) {
        if (s > s0) __syncthreads();   // the previous sub-item is done with the LDS
        auto kargs = __builtin_amdgcn_kernarg_segment_ptr();
        __asm__ volatile("" : "+s"(kargs));
        const BatchDev &B = *(const BatchDev *)kargs;
        Job J;
        J.f = f;
        J.P = ld_const(B.plans + f);
        J.io = io_of(B, f);
        J.local = s;
        switch (h) {
          case PH_PACK: pack_item<KIND>(B, J, lds, false); break;
          case PH_SPLITROWS: split_rows_item(B, J, reinterpret_cast<double *>(lds)); break;
          case PH_MOMENT:
            if constexpr (KIND == 0) moment_f64_item(B, J, reinterpret_cast<double *>(lds));
            else split_item<KIND, false>(B, J, reinterpret_cast<u4 *>(lds));
            break;
          case PH_REDUCE: reduce_item(J); break;
          case PH_SCAN: scan_item<PERSIST_SCAN_MODES>(J, reinterpret_cast<double *>(lds)); break;
          case PH_COEF:
            if constexpr (KIND == 0) perm_coef_item(J);
            else split_coef_item<KIND>(J, reinterpret_cast<double *>(lds));
            break;
          case PH_EXPAND:
            if constexpr (KIND == 0) expand_f64_item(B, J, reinterpret_cast<double *>(lds));
            else split_item<KIND, true>(B, J, reinterpret_cast<u4 *>(lds));
            break;
          case PH_BCAST: bcast_item(B, J); break;
          default: break;
        }
      }
      // the item's stores complete (in this XCD's L2) before it is counted
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
    if (h >= 0 && threadIdx.x == 0) {
      const PersistDev *qd = Qp;
      __asm__ volatile("" : "+v"(qd));
      atomicAdd(&qd->done[f * PH_COUNT + h], 1u);
    }
  }
}

// Per-solve reset of the dispensers, completion counters, error word and
// field completion stamps (a kernel, so that the solve can be captured).
__global__ __launch_bounds__(256) void k_persist_reset(PersistDev Q, unsigned long long *stamps, int nf) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < Q.nq) Q.next[t] = 0u;
  if (t < nf * PH_COUNT) Q.done[t] = 0u;
  if (t == 0) *Q.err = 0u;
  if (stamps != nullptr && t < nf) stamps[t] = 0ull;
  if (stamps != nullptr && t == nf) stamps[nf] = ~0ull;
}

// ids[w] = the XCD id workgroup w ran on.
__global__ __launch_bounds__(64) void k_xcc_probe(int32_t *ids) {
  if (threadIdx.x == 0) ids[blockIdx.x] = xcc_id();
}

template <int KIND>
int occupancy_blocks() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<KIND>, PERSIST_THREADS, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

}  // namespace

hipError_t launch_xcc_probe(int32_t *ids, int wgs, hipStream_t s) {
  hipLaunchKernelGGL(k_xcc_probe, dim3(wgs), dim3(64), 0, s, ids);
  return hipGetLastError();
}

int persistent_blocks_per_cu(int precision) {
  return precision == 0 ? occupancy_blocks<0>()
         : precision == kSplitBf16x3 ? occupancy_blocks<kSplitBf16x3>() : occupancy_blocks<kSplitFp16x2>();
}

int persistent_scan_modes() { return PERSIST_SCAN_MODES; }

hipError_t launch_persistent(const BatchDev &B, const PersistDev &Q, const PersistDev *Qdev, uint32_t spin_limit,
                             int precision, int grid, hipStream_t s) {
  const int n = std::max(Q.nq, B.nf * PH_COUNT + 1);
  hipLaunchKernelGGL(k_persist_reset, dim3((n + 255) / 256), dim3(256), 0, s, Q, B.stamps, B.nf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (precision == 0)
    hipLaunchKernelGGL(k_persistent<0>, dim3(grid), dim3(PERSIST_THREADS), 0, s, B, Qdev, spin_limit);
  else if (precision == kSplitBf16x3)
    hipLaunchKernelGGL(k_persistent<kSplitBf16x3>, dim3(grid), dim3(PERSIST_THREADS), 0, s, B, Qdev, spin_limit);
  else
    hipLaunchKernelGGL(k_persistent<kSplitFp16x2>, dim3(grid), dim3(PERSIST_THREADS), 0, s, B, Qdev, spin_limit);
  return hipGetLastError();
}

}  // namespace mpole
