// Device-visible description of one resultant job and of the global tables.
#pragma once
#include <stdint.h>

#include "modp.hpp"

namespace bires {

// One res(f, g; y) job after planning.  All pointers are device memory.
// f and g are dense rectangles of limbs (rows = powers of y); for a
// discriminant the g residues are formed from f (g_{j,i} = (j+1) f_{j+1,i}),
// for a polar resultant both operands are (f-side: (i+1) f_{j,i+1}, the
// x-derivative; g-side: the y-derivative).
struct JobDev {
  const uint32_t* limbs_f;  // [(m+1) * ldf * Lf]
  const uint32_t* limbs_g;  // [(n+1) * ldg * Lg]; unused unless kind == 0
  int32_t Lf, Lg;           // limbs per input coefficient
  int32_t ldf, ldg;         // row stride (coefficients) of the rectangles
  int32_t m, n;             // degrees in y (top non-zero row of f, g)
  int32_t kind;             // 0: g given; 1: g = df/dy; 2: f <- df/dx, g = df/dy
  int32_t P, D;             // primes, evaluation points (= degree bound + 1)
  int32_t lpf, lpg;         // row stride of the residue rows (ldf, ldg rounded up to 4)
  int32_t Tf, Tg;           // residues per prime: (m+1)*lpf, (n+1)*lpg; padding is zero
  const int32_t* rowdeg_f;  // [m+1] degree in x of each row (-1: zero row)
  const int32_t* rowdeg_g;  // [n+1]
  uint32_t* res_f;          // [P][Tf] Montgomery residues
  uint32_t* res_g;          // [P][Tg]
  uint32_t* vals;           // [P][D] values R(a) mod p_k, a = 0..D-1
  uint32_t* coefs;          // [P][D] coefficients of R mod p_k
  uint32_t* digits;         // [P][D] mixed-radix digits
  int32_t* negflag;         // [D] 1 when the symmetric lift is negative
  uint64_t* acc_lo;         // [Lacc][D] partial sums for limb assembly
  uint32_t* acc_hi;         // [Lacc][D]
  int32_t Lacc;             // min(Lcap, P + 1)
  uint32_t* out;            // [(degcap+1)][Lcap] result limbs
  int32_t Lcap, degcap;
  const uint32_t* crt;      // explicit CRT constants of the job's prime count (CrtHost layout)
  int32_t crt_LM;           // limbs of M = prod_{k<P} p_k
  int32_t* deg_out;         // highest non-zero coefficient index (init -1)
  int32_t* err;             // set non-zero on a failed internal check
  // jobs of the matrix-core interpolation group: the values go straight into
  // the group's digit planes (column ycol of ynp, ydp points per plane) instead
  // of vals; null otherwise
  int8_t* yp;
  int32_t ycol, ynp, ydp;
};

// One modular gcd over P primes (see k_gcd_p).
struct GcdDev {
  const uint32_t* res_a;  // [P][da+1] Montgomery residues of a
  const uint32_t* res_b;  // [P][db+1]
  int32_t da, db, P;
  const uint32_t* sc;     // [P][3] plain: beta, lc(a)/beta, lc(b)/beta mod p_k
  uint32_t* F;            // [P][dmin+1] beta * monic gcd mod p_k (plain), zero-padded
  uint32_t* QA;           // [P][da+1] (lc(a)/beta) * a / g mod p_k, zero-padded
  uint32_t* QB;           // [P][db+1] (lc(b)/beta) * b / g mod p_k
  int32_t* gdeg;          // [P] degree of the gcd mod p_k; -2: p_k divides lc(a) lc(b); -3: failed check
};

// The persistent fused launch (k_fused): every stage after the reduction (a
// launch of its own before it) for the whole batch in one launch of blocks of
// four waves, one stage after the other; the tasks of a stage are claimed in
// chunks from counters and a stage ends when all its tasks are done.  Wave
// tasks run on one wave and an LDS slice of its own: evaluation +
// elimination, the recomputation of the register-Euclid blocks that left the
// uniform case, the explicit CRT or the Garner digits, the limb carries.
// Block tasks run on the whole block: interpolation and the limb sums.
// Per-job first task of each stage as in the staged kernels.
constexpr int FUSED_STAGE_INTS = 512;  // counters of one stage of the fused launch

struct FusedPlan {
  const JobDev* jobs;
  int32_t nj;
  // evaluation + elimination: register Euclid (st_rg, n_rg blocks of 64
  // points), then the LDS kernel (st_ee, n_ee)
  const int* st_rg;
  const int* st_ee;
  int32_t n_rg, n_ee;
  int* fb_count;  // register-Euclid blocks queued for the LDS kernel (zero before the launch)
  int* fb_queue;  // [n_rg]
  // interpolation: on the matrix cores for a group sharing D and P (im = 1:
  // n_im blocks of 64 x 64), else per (job, prime) (st_ip, n_ip)
  int32_t im, n_im;
  uint32_t* const* gco;
  int32_t gN, gNp, gD, gDp;
  const int8_t* Ap;
  const int8_t* Yp;
  const int* st_ip;
  int32_t n_ip;
  const uint32_t* itW;  // Newton-to-monomial block tables (null: computed in place)
  const uint32_t* itQ;
  int32_t itNB;
  // reconstruction: explicit CRT (crt = 1: blocks of 32 rows) or Garner
  // digits, limb sums and limb carries
  int32_t crt;
  const int* st_crt;
  int32_t n_crt, sld, cps;
  const int* st_mrc;
  int32_t n_mrc;
  const int* st_sum;
  int32_t n_sum;
  const int* st_car;
  int32_t n_car, stage_ld;
  // per wave stage (0 evaluation, 1 recomputation, 2 CRT or digits, 3
  // carries): the waves of a block that take its tasks, the words of a
  // wave's LDS slice
  int32_t wv[4], lw[4];
  // tasks per claim of stages 0 evaluation, 1 (one), 2 interpolation, 3 CRT
  // or digits, 4 limb sums, 5 carries
  int32_t kc[6];
  int* ctr;  // [6][FUSED_STAGE_INTS]: per stage claim heads and finished-task counts (zero before the launch)
  int* err;  // bit 1: a wait timed out
};

// The degree chain of the N^- / N^+ test over one prime (k_fiber_chain).
struct ChainDev {
  const uint32_t* rstar;  // [dr + 1] R* mod p (Montgomery)
  int32_t dr;             // its extent (leading coefficient may vanish mod p)
  const uint32_t* srs;    // [K][D] sr_i mod p (plain), rows 1..K-1 used
  int32_t K, D;
  const uint32_t* qpol;   // [Dq] Q mod p (plain)
  int32_t Dq;
  int32_t* out;           // [K + 2]: deg S_0 .. deg S_{K-1} (0 past the end), deg gcd(R^inf, Q), Q mod p = 0
};

// Tables shared by every job: the prime list and the mixed-radix constants.
struct TablesDev {
  const ModP* primes;       // [K]
  const uint32_t* gm;       // [K][K]: gm[j*K+k] = (prod_{i<j} p_i) R mod p_k, j < k
  const uint32_t* cm;       // [K]: (prod_{i<k} p_i)^{-1} R mod p_k
  const uint32_t* pm;       // [K][K]: pm[k*K+j] = (p_j mod p_k) R mod p_k, j < k
  const uint32_t* pi;       // prod_{i<k} p_i as k+1 limbs at offset k(k+1)/2
  const uint32_t* invfact;  // [K][dmax]: Montgomery form of 1/n! mod p_k
  const double* inv_p;      // [K]: 1 / p_k rounded to nearest
  int32_t K;
  int32_t dmax;
};

}  // namespace bires
