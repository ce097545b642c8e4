// Launchers of the HIP kernels in kernels.hip (host-callable, no HIP types
// beyond hipStream_t and the plain structs of job.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include "job.hpp"

namespace bires {

// Planning statistics of one limb rectangle: out[3*j + {0,1,2}] =
// (x-degree of row j or -1, max bit length of |c| in the row, non-zero count).
struct ScanTask {
  const uint32_t* limbs;
  int32_t rows, ld, L;
  int32_t* out;
};

void launch_scan(const ScanTask* tasks, const int4* bmap, int nblocks, hipStream_t s);
// Issue-rate probe: kind 0..5 = v_add_u32, v_min_u32, v_mul_lo_u32,
// v_mad_u64_u32, v_fma_f64 (16 chains per lane), v_mfma_i32_32x32x32_i8
// (16 products per round over 4 accumulators); `iters` rounds; out holds
// blocks * 256 words.
void launch_issue_rate(int kind, uint32_t* out, int blocks, int iters, hipStream_t s);
// Sets *flag (not cleared here) when got[0..n) and want[0..n) differ.
void launch_stats_check(const int32_t* got, const int32_t* want, long long n, int* flag, hipStream_t s);
// dst[0..words) = src_mapped[0..words): src_mapped is the device mapping of
// pinned host memory (hipHostGetDevicePointer).
void launch_upload(const uint32_t* src_mapped, uint32_t* dst, long long words, hipStream_t s);
void launch_transpose(const uint32_t* src, uint32_t* dst, int rows, int cols, int L, hipStream_t s);
// Job launchers: starts[0..nj] hold the first block of each job (starts[nj] = nblocks).
// Blocks per job: reduce ceil(Tf/64)+ceil(Tg/64); eval_elim P*ceil(D/64);
// interp P; mrc D; limbs_sum ceil(D*Lacc/256); limbs_carry ceil((degcap+1)/64).
void launch_reduce(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_primes, TablesDev tab,
                   hipStream_t s);
int eval_elim_block();
// Residue rows are stored at a stride rounded up to a multiple of 4 words so
// the evaluation reads them as aligned 16-byte groups.
inline int pad4(int ld) { return (ld + 3) & ~3; }
// max_words: max over jobs of m+n+2; max_res: max over jobs of Tf+Tg (padded).
size_t eval_elim_lds_bytes(int words, int res);
void launch_eval_elim(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_words, int max_res,
                      TablesDev tab, hipStream_t s);
// Evaluation + elimination with f's coefficient array in registers: the
// register capacity C (24, 32 or 64) for a job of degrees m, n in the
// eliminated variable, or 0 when the job needs the LDS kernel (min(m, n) = 0
// or max(m, n) >= 64).  launch_eval_elim_rg runs the blocks of jobs with that
// capacity (max_deg = max over jobs of max(m, n), max_words of m + n + 2),
// then recomputes with launch_eval_elim's kernel the blocks that leave the
// uniform normal case.  fb_count: one device int, zero before the launch;
// fb_queue: nblocks ints of workspace.
int eval_elim_rg_capacity(int m, int n);
void launch_eval_elim_rg(int C, const JobDev* jobs, const int* starts, int nj, int nblocks, int max_deg,
                         int max_words, int* fb_count, int* fb_queue, TablesDev tab, hipStream_t s);
// Evaluation + elimination by the Schur algorithm on the displacement
// generators, one wave (block of 64) per (prime, point) instance: P * D blocks
// per job; rows per lane NR = schur_rows_per_lane(m, n) (0: the job cannot
// use it: min(m, n) = 0 or m + n > 128); max_words: max over jobs of m + n + 2.
int schur_rows_per_lane(int m, int n);
// fallbacks: one device int counting the instances recomputed by Euclid.
void launch_schur(int NR, const JobDev* jobs, const int* starts, int nj, int nblocks, int max_words, int* fallbacks,
                  TablesDev tab, hipStream_t s);
// Interpolation of one (job, prime) per block.  W, Q: the block tables of
// launch_interp_tables for tab_blocks blocks (null: computed in the kernel).
void launch_interp(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_points, TablesDev tab,
                   const uint32_t* W, const uint32_t* Q, int tab_blocks, hipStream_t s);
// Newton-to-monomial block tables for `blocks` 32-node blocks (enough for
// max_points nodes: interp_table_blocks) and the first `primes` primes:
// interp_table_words words, W at 0 and Q at *q_offset.
int interp_table_blocks(int max_points);
size_t interp_table_words(int blocks, int primes, size_t* q_offset);
void launch_interp_tables(int blocks, int primes, TablesDev tab, uint32_t* W, uint32_t* Q, hipStream_t s);
size_t interp_lds_words(int D);
// Interpolation of N jobs sharing D and P (gco[n] the coefs of job n of the
// group) as int8 matrix-core products with V^{-1}: Ap = vinv_bytes(Dp, P)
// bytes built by launch_vinv (Dp = D rounded up to 32); Yp = 4 Np Dp P bytes
// (Np = N rounded up to 32) holding the jobs' values as digit planes, which
// the evaluation kernels write (JobDev::yp).  Writes the jobs' coefs.
size_t vinv_bytes(int Dp, int P);
void launch_vinv(int D, int Dp, int P, TablesDev tab, int8_t* Ap, hipStream_t s);
void launch_interp_mfma(uint32_t* const* gco, int N, int D, int P, const int8_t* Ap, const int8_t* Yp, TablesDev tab,
                        hipStream_t s);
void launch_invfact(const ModP* primes, int K, uint32_t* invfact, int dmax, hipStream_t s);
// Garner digits: one wave per coefficient, D blocks per job.
void launch_mrc(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_primes, TablesDev tab,
                hipStream_t s);
// Explicit CRT straight to limbs on the matrix cores (k_crt_mfma): one wave
// per rows = crt_rows_per_block(max primes) output coefficients,
// ceil(min(D, degcap + 1) / rows) blocks per job, which also write the job's
// zero coefficients above them up to degcap; needs crt_ok(max primes), the
// jobs' crt tables (crt_tables layout) and crt_lds_bytes(max output limbs,
// max primes) within the LDS per block.
bool crt_ok(int max_primes);
size_t crt_lds_bytes(int max_lcap, int max_primes);
size_t crt_lds_bytes_rows(int max_lcap, int max_primes, int rows);
// the CRT's LDS strides: limb rows (sld) and prime constants (cps)
int crt_row_stride(int max_lcap);
int crt_const_stride(int max_primes);
int crt_rows_per_block(int max_primes);
void launch_crt(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_primes, int max_lcap,
                TablesDev tab, hipStream_t s);
void launch_limbs_sum(const JobDev* jobs, const int* starts, int nj, int nblocks, TablesDev tab, hipStream_t s);
// Persistent fused launch (see FusedPlan), blocks of 256 threads: C the
// register Euclid's capacity (fused_capacity: 24, 32, or 0 for the LDS
// kernel only), KS = fused_crt_steps(max primes); blocks of one CU at once
// for this LDS size (0 on a runtime error).  The matrix-core interpolation
// takes fused_interp_lds_bytes per block (64 x 32 blocks of C), the CRT
// crt_lds_bytes_rows(.., 32) per wave.
int fused_capacity(int rg_capacity);
int fused_crt_steps(int max_primes);
int fused_blocks_per_cu(int C, int KS, size_t lds_bytes);
size_t fused_interp_lds_bytes();
void launch_fused(int C, int KS, const FusedPlan& F, size_t lds_bytes, int blocks, TablesDev tab, hipStream_t s);
// Principal subresultant coefficients modulo prime index 0 of tab (the caller
// shifts the table to its prime): one lane per point a < J.D, J.m and J.n the
// formal degrees; writes sr_i(a) (plain) to num[i * D + a] for i < K, with
// den ([K][D]) as workspace.
size_t psc_lds_bytes(int m, int n);
void launch_psc(const JobDev& J, TablesDev tab, uint32_t* num, uint32_t* den, int K, hipStream_t s);
// The N^- / N^+ degree chain over prime index 0 of tab, one block.
size_t fiber_chain_lds_bytes(int dr, int D, int Dq);
void launch_fiber_chain(const ChainDev& C, TablesDev tab, hipStream_t s);
size_t gcd_lds_bytes(int da, int db);
void launch_gcd_p(const GcdDev& g, TablesDev tab, hipStream_t s);
void launch_gather_rows(const uint32_t* src, int ld, const int* idx, int rows, int n, uint32_t* dst, hipStream_t s);
// max_lcap: the largest Lcap of the jobs in the launch.
void launch_limbs_carry(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_lcap, hipStream_t s);

}  // namespace bires
