// Basis update in double-double for blocks of 9 to 64 columns: the DD
// result of one pass (Sec. 4.2: kernels that return double-double results),
// Q + Q_lo = (S + S_lo - Y (C + C_lo)) (Z + Z_lo) rounded once per entry.
//
// The arithmetic is that of the narrow kernel's DD branch (update_narrow.hpp),
// in the same order: each entry of T = S - Y C starts from S (and the low
// word of a DD input) and takes the products y C_hi with the Dot2 step and
// y C_lo into its error term; each entry of Q sums t_hi Z_hi with the Dot2
// step and t_hi Z_lo + t_lo Z_hi into its error term, over l = 0, 1, ... (l
// <= j for triangular Z, all l for SVQB's dense Z), and is rounded by TwoSum.
// With more than eight columns T no longer fits a lane's registers, so each
// lane keeps its row of T (hi and lo words) in LDS; no lane reads another's,
// so the LDS needs no barrier.  One wave per workgroup, one row per lane,
// 64-row panels in a grid-stride loop; T and Q are worked in chunks of eight
// columns.  C and Z are the same for every lane and are read through the
// scalar cache.  The sweep is bound by the FP64 vector ALUs (about 10
// instructions per product), not by HBM.
#include <mutex>

#include "dd.hpp"
#include "internal.hpp"

namespace borth {
namespace {

template <int KN>
__global__ void __launch_bounds__(64) dd_update_kernel(UpdDev a, int kp) {
  extern __shared__ double lds_t[];
  if (stopped(a.stop, a.pass)) return;
  constexpr int SP = KN + 1;  // odd row stride
  double* Th = lds_t;
  double* Tl = lds_t + 64 * SP;
  const int lane = threadIdx.x;
  const int ky = a.ky, k = a.k;
  const int64_t m = a.m;
  typedef const double __attribute__((address_space(4)))* cptr;
  const cptr Cg = (cptr)a.C1;
  const cptr Clg = (cptr)a.C1lo;
  const cptr Zg = (cptr)a.Z1;
  const cptr Zlg = (cptr)a.Z1lo;
  const double BORTH_GLOBAL* __restrict__ Xg = gmem((const double*)a.X);
  const double BORTH_GLOBAL* __restrict__ Xlg = gmem(a.Xlo);
  const double BORTH_GLOBAL* __restrict__ Yg = gmem(a.Y);
  double BORTH_GLOBAL* __restrict__ Qg = gmem(a.Q);
  double BORTH_GLOBAL* __restrict__ Qlg = gmem(a.Qlo);
  const int64_t npanels = (m + 63) / 64;
  for (int64_t p = blockIdx.x; p < npanels; p += gridDim.x) {
    const int64_t row0 = p * 64;
    const int nrows = (int)(m - row0 < 64 ? m - row0 : 64);
    const bool live = lane < nrows;
    const int64_t row = row0 + (live ? lane : nrows - 1);  // rows past m: the last row, not stored
    // T = S - Y C, eight columns at a time
#pragma unroll 1
    for (int jc = 0; jc < k; jc += 8) {
      double ts[8], te[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int j = jc + jj;
        ts[jj] = j < k ? Xg[row * a.ldx + j] : 0.0;
        te[jj] = (Xlg && j < k) ? Xlg[row * a.ldx + j] : 0.0;
      }
#pragma unroll 2
      for (int c = 0; c < ky; ++c) {
        const double y = Yg[row * a.ldy + c];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          dot2_step(ts[jj], te[jj], y, -Cg[c * kp + jc + jj]);
          te[jj] = __builtin_fma(y, -Clg[c * kp + jc + jj], te[jj]);
        }
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        Th[lane * SP + jc + jj] = ts[jj];
        Tl[lane * SP + jc + jj] = te[jj];
      }
    }
    // Q = T Z, eight columns at a time
#pragma unroll 1
    for (int jc = 0; jc < k; jc += 8) {
      double s[8], e[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) s[jj] = e[jj] = 0.0;
      const int lend = a.dense ? k : (jc + 8 < k ? jc + 8 : k);
#pragma unroll 1
      for (int l = 0; l < lend; ++l) {
        const double th = Th[lane * SP + l], tl = Tl[lane * SP + l];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          if (a.dense || l <= jc + jj) {  // Z upper triangular unless dense
            const double zh = Zg[l * kp + jc + jj];
            dot2_step(s[jj], e[jj], th, zh);
            e[jj] = __builtin_fma(th, Zlg[l * kp + jc + jj], __builtin_fma(tl, zh, e[jj]));
          }
        }
      }
      if (live) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          const int j = jc + jj;
          if (j < k) {
            const dd_t q = two_sum(s[jj], e[jj]);
            Qg[row * a.ldq + j] = q.hi;
            Qlg[row * a.ldq + j] = q.lo;
          }
        }
      }
    }
  }
}

template <int KN>
hipError_t launch_kn(const UpdDev& d, int kp, hipStream_t st) {
  const size_t shmem = sizeof(double) * 2 * 64 * (KN + 1);
  static std::once_flag attr;
  std::call_once(attr, [shmem] {
    (void)hipFuncSetAttribute((const void*)dd_update_kernel<KN>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  });
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, dd_update_kernel<KN>, 64, shmem) != hipSuccess ||
      per < 1)
    return hipErrorInvalidConfiguration;
  int64_t grid = (d.m + 63) / 64;
  if (grid > (int64_t)per * cus) grid = (int64_t)per * cus;
  if (grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dd_update_kernel<KN>), dim3((unsigned)grid), dim3(64), shmem, st, d, kp);
  return hipGetLastError();
}

}  // namespace

bool update_dd_ok(int k, int ky, int kp) {
  return k > 8 && k <= 64 && ky >= 0 && ky <= 64 && kp >= k && kp <= 64;
}

hipError_t launch_update_dd(const UpdDev& d, int kp, hipStream_t st) {
  if (!update_dd_ok(d.k, d.ky, kp) || d.m < 1 || !d.Q || !d.Qlo || !d.C1 || !d.Z1 || !d.C1lo ||
      !d.Z1lo)
    return hipErrorInvalidValue;
  if (d.k <= 16) return launch_kn<16>(d, kp, st);
  if (d.k <= 32) return launch_kn<32>(d, kp, st);
  return launch_kn<64>(d, kp, st);
}

}  // namespace borth
