// Segmented vector kernels of the optimiser (internal).
#pragma once
#include "common.hpp"

namespace tlr {

// A contiguous run of at most VEC_CH floats belonging to one problem.
struct VecSeg {
    int64_t off;    // first float
    int32_t n;      // floats in the run
    int32_t prob;   // problem index
    int32_t part;   // partial-sum slot (prob * pstride + local index)
    int32_t pad;
};
constexpr int VEC_CH = 4096;   // floats per segment (a multiple of 1024; offsets multiples of 4)

enum FinOp : int32_t {
    FIN_INIT = 0, FIN_F, FIN_F_OUT, FIN_THNORM, FIN_GRAM, FIN_LAMTERMS, FIN_LINE, FIN_RECORD, FIN_RESET
};

struct FinArgs {
    int32_t op;
    int32_t nsum;          // sums per partial entry
    const double *partials;
    int64_t pstride;       // entries per problem
    const int32_t *counts; // entries used per problem (NULL -> ucount)
    int32_t ucount;
    int32_t m1;            // ring slots (lbfgs_m + 1)
    int32_t t;             // f-history index (FIN_F)
    SolveScalars *sc;
    double *const *fhist;  // device table of per-problem f-history pointers (FIN_F, batches)
    double *fhist0;        // f-history of a single problem (FIN_F)
    double *fout;          // FIN_F_OUT: per-problem objective
    double lam;
    double *gram;          // FIN_GRAM: per-problem Gram matrix and direction coefficients
    int64_t gstride;       // doubles per problem in gram: (2 m1 + 1)^2 + 2 m1 + 1
};

hipError_t launch_gram(const VecSeg *segs, int nseg, int m1, const float *g, const float *gprev, float *Yb,
                       const float *Sb, int64_t stride2, const SolveScalars *sc, double *part, hipStream_t s);
hipError_t launch_combine(const VecSeg *segs, int nseg, int m1, float *p, const float *g, const float *Sb,
                          const float *Yb, int64_t stride2, const SolveScalars *sc, const double *coef,
                          int64_t cstride, hipStream_t s);
hipError_t launch_negate(const VecSeg *segs, int nseg, float *p, const float *g, hipStream_t s);
hipError_t launch_reg_grad(const VecSeg *segs, int nseg, float *g, const float *th, const float *cen, float lam2,
                           hipStream_t s);
hipError_t launch_pen(const VecSeg *segs, int nseg, const float *th, const float *cen, const float *p, double *part,
                      hipStream_t s);
hipError_t launch_admm_update(const VecSeg *segs, int nseg, int init, const float *th, float *z, float *u, float *cen,
                              float scale, hipStream_t s);
hipError_t launch_theta_update(const VecSeg *segs, int nseg, float *th, const float *p, float *Sb,
                               int64_t stride2, const float *cen, const SolveScalars *sc, double *part,
                               hipStream_t s);
hipError_t launch_resid_update(const VecSeg *segs, int nseg, float *r, const float *a, const float *b,
                               const SolveScalars *sc, double *part, hipStream_t s);
hipError_t launch_finalize(const FinArgs &fa, int nprob, hipStream_t s);

}  // namespace tlr
