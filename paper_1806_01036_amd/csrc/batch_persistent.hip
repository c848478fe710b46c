// Persistent batched kernel: see batch_persist.hpp for the design.  The task
// bodies are those of the per-phase kernels (gram_impl.hpp, update_impl.hpp,
// factor_impl.hpp), so a block's arithmetic is the same in both drivers; the
// k x k step runs on 16 x 16 threads with its working arrays in global
// memory (the LDS belongs to the sweeps), and the reduction of partial sums
// adds them in the order of the reduction kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "batch_persist.hpp"
#include "dd.hpp"
#include "factor_impl.hpp"
#include "gram_impl.hpp"
#include "update_impl.hpp"

namespace borth {
namespace {

// Pauses (s_sleep 32: about 1 us each) before an idle workgroup leaves while
// blocks are still unfinished: long enough to outlast any gap between sweeps
// (a k x k step takes well under a millisecond), short enough that a
// workgroup can never hold the device for long.
constexpr int kMaxIdle = 200000;

// Offsets (doubles) in a workgroup's global working memory.
constexpr int64_t kFmR0 = 0, kFmR1 = 2 * 64 * 65, kFmRow = 4 * 64 * 65, kFmPiv = kFmRow + 256,
                  kFmFlag = kFmPiv + 128, kFmMsg = kFmFlag + 8, kFmDinv = kFmMsg + 8;
static_assert(kFmDinv + 4 <= kPersistFactorDoubles, "factor working memory");

// Each task body is a function of its own (not inlined into the kernel), so
// that the register allocator treats it as it treats that body's own
// kernel: inlined into one kernel, every body shared the kernel's register
// budget with the others and spilled inside its loops.
template <int K, int KYP, int GR>
__device__ __attribute__((noinline)) void run_update_v(const PSweep& sw, int bid, double* pool) {
  const UpdDev* tab = (const UpdDev*)sw.tab;
  upd::update_body<K, KYP, false, GR, double, true, false>(tab[0], tab, sw.map, bid, sw.nw, pool);
}

template <int K>
__device__ __forceinline__ void run_update_k(const PSweep& sw, int bid, double* pool) {
  if (sw.KYP == 16 && sw.GR == 2)
    run_update_v<K, 16, 2>(sw, bid, pool);
  else if (sw.KYP == 16)
    run_update_v<K, 16, 0>(sw, bid, pool);
  else if (sw.GR == 1)
    run_update_v<K, 0, 1>(sw, bid, pool);
  else
    run_update_v<K, 0, 0>(sw, bid, pool);
}

__device__ __attribute__((noinline)) void run_gram_dma(const PSweep& sw, int bid, double* pool) {
  const GramSeg* tab = (const GramSeg*)sw.tab;
  gram_dd_dma_body<true, true, 0>(tab[0], tab, sw.map, bid, pool);
}

__device__ __attribute__((noinline)) void run_gram_tiles(const PSweep& sw, int bid, double* pool) {
  const GramSeg* tab = (const GramSeg*)sw.tab;
  gram_tiles_body<true, 256, true, false>(tab[0], tab, sw.map, bid, pool);
}

__device__ __forceinline__ void run_sweep(const PSweep& sw, int bid, double* pool) {
  if (sw.kind == 0) {
    run_gram_dma(sw, bid, pool);
  } else if (sw.kind == 1) {
    run_gram_tiles(sw, bid, pool);
  } else {
    switch (sw.K) {
      case 8: run_update_k<8>(sw, bid, pool); break;
      case 16: run_update_k<16>(sw, bid, pool); break;
      case 32: run_update_k<32>(sw, bid, pool); break;
      default: run_update_k<64>(sw, bid, pool); break;
    }
  }
}

template <bool DD>
__device__ __attribute__((noinline)) void run_reduce(const ReduceSeg& rs) {
  reduce_segment_body<DD>(rs);
}

template <bool DD, int NS>
__device__ __attribute__((noinline)) void run_chol_v(const FactorArgs& fa, const fct::CholMem& mem) {
  fct::chol_body<DD, 16, NS>(fa, mem);
}

template <bool DD>
__device__ __forceinline__ void run_chol(const FactorArgs& fa, int ns, const fct::CholMem& mem) {
  if (ns == 1)
    run_chol_v<DD, 1>(fa, mem);
  else if (ns == 2)
    run_chol_v<DD, 2>(fa, mem);
  else
    run_chol_v<DD, 4>(fa, mem);
}

// State (ints, set by batch_init_kernel before every launch):
//   claimed[3 nb], done[3 nb]  shares taken / finished per (block, sweep)
//   finished                   blocks finished
//   qtail                      sweeps opened (queue entries reserved)
//   qhead                      a queue position before which every opened
//                              sweep's shares are all taken
//   queue[3 nb]                opened sweeps in the order they opened, as
//                              4 b + s (-1 while reserved and not written);
//                              the first nb are the blocks' Gram sweeps,
//                              larger blocks first
constexpr int kStClaimed = 0;
__host__ __device__ inline int st_done(int nb) { return 3 * nb; }
__host__ __device__ inline int st_finished(int nb) { return 6 * nb; }
__host__ __device__ inline int st_qtail(int nb) { return 6 * nb + 1; }
__host__ __device__ inline int st_qhead(int nb) { return 6 * nb + 2; }
__host__ __device__ inline int st_queue(int nb) { return 6 * nb + 3; }

__global__ void batch_init_kernel(int* state, const int* __restrict__ order, int nb) {
  const int n = 9 * nb + 3;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int v = 0;
    if (i == st_qtail(nb)) v = nb;
    if (i >= st_queue(nb)) {
      const int q = i - st_queue(nb);
      v = q < nb ? 4 * order[q] : -1;
    }
    state[i] = v;
  }
}

__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256, 2) batch_persistent_kernel(const PBlock* __restrict__ blocks,
                                                                  int nb, int* state,
                                                                  double* scratch) {
  extern __shared__ double pool[];
  int* claimed = state + kStClaimed;
  int* done = state + st_done(nb);
  int* finished = state + st_finished(nb);
  int* qtail = state + st_qtail(nb);
  int* qhead = state + st_qhead(nb);
  int* queue = state + st_queue(nb);
  double* fm = scratch + (int64_t)blockIdx.x * kPersistFactorDoubles;
  // messages from thread 0 to the workgroup (global memory, read after a
  // barrier: the workgroup's waves share the compute unit's cache)
  volatile int* msg = (volatile int*)(fm + kFmMsg);
  const fct::CholMem mem{fm + kFmR0, fm + kFmR1, fm + kFmRow, fm + kFmPiv, (int*)(fm + kFmFlag),
                         fm + kFmDinv};
  const int tid = threadIdx.x;
  int idle = 0;
  for (;;) {
    if (tid == 0) {
      // the oldest opened sweep with a share left: walk the queue from its
      // head, moving the head past sweeps whose shares are all taken
      int fb = -1, fs = 0, fu = 0;
      int q = ld_relaxed(qhead);
      const int tail = ld_relaxed(qtail);
      bool prefix = true;  // every entry before q is exhausted
      while (q < tail && fb < 0) {
        const int e = ld_relaxed(&queue[q]);
        if (e < 0) {  // reserved, not yet written: skip for now
          prefix = false;
          ++q;
          continue;
        }
        const int b = e >> 2, sw = e & 3;
        const int n = blocks[b].sw[sw].ntasks;
        int* cl = &claimed[3 * b + sw];
        if (ld_relaxed(cl) < n) {
          const int u = atomicAdd(cl, 1);
          if (u < n) {
            fb = b;
            fs = sw;
            fu = u;
            break;
          }
        }
        ++q;
        if (prefix) atomicMax(qhead, q);
      }
      const int fin = fb < 0 ? ld_relaxed(finished) : 0;
      // acquire: what the sweep's opener and the block's earlier sweeps wrote
      __threadfence();
      msg[0] = fb;
      msg[1] = fs;
      msg[2] = fu;
      msg[3] = fin;
    }
    __syncthreads();
    const int b = msg[0], s = msg[1], u = msg[2], fin = msg[3];
    __syncthreads();
    if (b < 0) {
      if (fin >= nb || ++idle > kMaxIdle) break;
      __builtin_amdgcn_s_sleep(32);
      continue;
    }
    idle = 0;
    const PSweep& sw = blocks[b].sw[s];
    run_sweep(sw, sw.wg0 + u, pool);
    __syncthreads();
    if (tid == 0) {
      __threadfence();  // release this share's partial sums / rows of Q
      const int d = atomicAdd(&done[3 * b + s], 1);
      const int last = d == sw.ntasks - 1 ? 1 : 0;
      if (last) __threadfence();  // acquire every share of the sweep
      msg[0] = last;
    }
    __syncthreads();
    const int last = msg[0];
    __syncthreads();
    if (!last) continue;
    // the last share of block b's sweep s: its reduction and k x k step,
    // then the block's next sweep opens at the queue's tail
    const PBlock& B = blocks[b];
    if (s + 1 < B.nsweeps) {
      if (B.red_dd[s])
        run_reduce<true>(B.red[s]);
      else
        run_reduce<false>(B.red[s]);
      __syncthreads();
      if (B.fac[s].dd)
        run_chol<true>(B.fac[s], B.fac_ns[s], mem);
      else
        run_chol<false>(B.fac[s], B.fac_ns[s], mem);
      __syncthreads();
    }
    if (tid == 0) {
      __threadfence();  // release the block's k x k results and its sweep
      if (s + 1 < B.nsweeps) {
        const int q = atomicAdd(qtail, 1);
        __hip_atomic_store(&queue[q], 4 * b + s + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        atomicAdd(finished, 1);
      }
    }
    __syncthreads();
  }
}

}  // namespace

bool persist_update_ok(int K, int KYP, int GR) {
  if (K != 8 && K != 16 && K != 32 && K != 64) return false;
  return (KYP == 16 && (GR == 2 || GR == 0)) || (KYP == 0 && (GR == 1 || GR == 0));
}

int persist_update_waves(int K, int KYP, int GR) {
  if (!persist_update_ok(K, KYP, GR)) return 0;
  const int KC = (K + 15) / 16, T16 = (GR == 2 ? 1 : 0) + KC;
  const long red = GR ? 8L * T16 * (T16 + 1) / 2 * 4 * 64 : 0;
  for (int nw = 4; nw >= 1; --nw) {
    long b = upd::upd_lds_bytes(K, KYP, nw, 1, false);
    if (red > b) b = red;
    if (b <= (long)kPersistLds) return nw;
  }
  return 0;
}

int batch_persistent_grid() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  static std::once_flag attr;
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute((const void*)batch_persistent_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPersistLds);
  });
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_persistent_kernel, 256, kPersistLds) !=
          hipSuccess)
    return 0;
  return per * cus;
}

int batch_persistent_state_ints(int nb) { return 9 * nb + 3; }

hipError_t launch_batch_persistent(const PBlock* blocks, const int* order, int nb, int* state,
                                   double* scratch, int grid, hipStream_t st) {
  if (nb < 1 || grid < 1 || !blocks || !order || !state || !scratch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_init_kernel, dim3((9 * nb + 3 + 255) / 256), dim3(256), 0, st, state,
                     order, nb);
  hipLaunchKernelGGL(batch_persistent_kernel, dim3(grid), dim3(256), kPersistLds, st, blocks, nb,
                     state, scratch);
  return hipGetLastError();
}

}  // namespace borth
