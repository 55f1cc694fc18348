// ctu_dispatch.hpp -- selection of the kernel instantiation for an option set.
//
// The sweep and Godunov kernels are templates over the direction, the
// physics, the predictor, the reconstruction kind and the Riemann solver, so
// that each supported combination compiles to straight-line code.  The
// instantiations are spread over one translation unit per precision.
#pragma once
#include "ctu_kernels.hpp"

namespace ctu {

struct Combo {
    int phys, pred, rk, rs;
    int shk;   // App. B shock flags in use
    int fast;  // options equal the fast variant's fixed set (see variant_opts)
    int par;   // ... the par variant's: the fast set with parabolic terms or cooling
};

// supported (physics, predictor, reconstruction, solver) combinations
__host__ inline bool combo_supported(const Combo &c)
{
    // c.phys: PHYS_MHD, PHYS_RMHD or PHYS_RMHD_TM (RMHD with the TM EOS)
    if (c.phys == PHYS_MHD) {
        if (c.pred == PRED_CHAR) return true;
        return c.rk == RK_LIN;
    }
    return c.pred == PRED_MH && c.rk == RK_LIN &&
           (c.rs == RS_HLL || c.rs == RS_RUSANOV || c.rs == RS_HLLC || c.rs == RS_HLLD);
}

hipError_t launch_sweep_f32(int D, const Combo &c, int nblocks, const SweepArgs<float> &a, hipStream_t s);
hipError_t launch_sweep_f64(int D, const Combo &c, int nblocks, const SweepArgs<double> &a, hipStream_t s);
hipError_t launch_mtflux_f32(int D, const Combo &c, int nblocks, const MtArgs<float> &a, hipStream_t s);
hipError_t launch_mtflux_f64(int D, const Combo &c, int nblocks, const MtArgs<double> &a, hipStream_t s);
hipError_t launch_tcouple_f32(int dim, int par, const Combo &c, int nblocks, const TArgs<float> &a, hipStream_t s);
hipError_t launch_tcouple_f64(int dim, int par, const Combo &c, int nblocks, const TArgs<double> &a, hipStream_t s);
// div != 0: k_pdiv (Pi^n divergence), else k_pflux (Pi^{n+1/2} face slots)
hipError_t launch_pflux_f32(int dim, int div, int nblocks, const PArgs<float> &a, hipStream_t s);
hipError_t launch_pflux_f64(int dim, int div, int nblocks, const PArgs<double> &a, hipStream_t s);

template <typename R> inline hipError_t launch_sweep(int D, const Combo &c, int nb, const SweepArgs<R> &a, hipStream_t s);
template <> inline hipError_t launch_sweep<float>(int D, const Combo &c, int nb, const SweepArgs<float> &a, hipStream_t s)
{
    return launch_sweep_f32(D, c, nb, a, s);
}
template <> inline hipError_t launch_sweep<double>(int D, const Combo &c, int nb, const SweepArgs<double> &a, hipStream_t s)
{
    return launch_sweep_f64(D, c, nb, a, s);
}

}  // namespace ctu

// Body of one precision's dispatch translation unit.
#define CTU_DEFINE_DISPATCH(R, SUFFIX)                                                                            \
    namespace ctu {                                                                                              \
    template <int D, int PHYS, int PRED, int RK, int RS, int VAR>                                                \
    static hipError_t sweep_one2(int nb, const SweepArgs<R> &a, hipStream_t s)                                  \
    {                                                                                                            \
        hipLaunchKernelGGL((k_sweep<D, PHYS, PRED, RK, RS, VAR, R>), dim3(nb), dim3(NT), 0, s, a);             \
        return hipGetLastError();                                                                                \
    }                                                                                                            \
    template <int D, int PHYS, int PRED, int RK, int RS>                                                         \
    static hipError_t sweep_one(const Combo &c, int nb, const SweepArgs<R> &a, hipStream_t s)                   \
    {                                                                                                            \
        /* Rusanov, HLLC and Roe have no hybrid-flag variant; parabolic terms  \
           and cooling belong to the MHD module */                                                               \
        if constexpr (RS != RS_RUSANOV && RS != RS_HLLC && RS != RS_ROE)                                         \
            if (a.flag) return sweep_one2<D, PHYS, PRED, RK, RS, VAR_SHOCK>(nb, a, s);                           \
        if (c.fast) return sweep_one2<D, PHYS, PRED, RK, RS, VAR_FAST>(nb, a, s);                                \
        if constexpr (PHYS == PHYS_MHD)                                                                          \
            if (c.par) return sweep_one2<D, PHYS, PRED, RK, RS, VAR_PAR>(nb, a, s);                              \
        return sweep_one2<D, PHYS, PRED, RK, RS, VAR_GENERIC>(nb, a, s);                                         \
    }                                                                                                            \
    template <int D>                                                                                             \
    static hipError_t sweep_dir(const Combo &c, int nb, const SweepArgs<R> &a, hipStream_t s)                   \
    {                                                                                                            \
        if (c.phys == PHYS_RMHD) {                                                                               \
            if (c.rs == RS_RUSANOV) return sweep_one<D, PHYS_RMHD, PRED_MH, RK_LIN, RS_RUSANOV>(c, nb, a, s);     \
            if (c.rs == RS_HLLC) return sweep_one<D, PHYS_RMHD, PRED_MH, RK_LIN, RS_HLLC>(c, nb, a, s);           \
            if (c.rs == RS_HLLD) return sweep_one<D, PHYS_RMHD, PRED_MH, RK_LIN, RS_HLLD>(c, nb, a, s);           \
            return sweep_one<D, PHYS_RMHD, PRED_MH, RK_LIN, RS_HLL>(c, nb, a, s);                                 \
        }                                                                                                        \
        if (c.phys == PHYS_RMHD_TM) {                                                                            \
            if (c.rs == RS_RUSANOV) return sweep_one<D, PHYS_RMHD_TM, PRED_MH, RK_LIN, RS_RUSANOV>(c, nb, a, s);  \
            if (c.rs == RS_HLLC) return sweep_one<D, PHYS_RMHD_TM, PRED_MH, RK_LIN, RS_HLLC>(c, nb, a, s);        \
            if (c.rs == RS_HLLD) return sweep_one<D, PHYS_RMHD_TM, PRED_MH, RK_LIN, RS_HLLD>(c, nb, a, s);        \
            return sweep_one<D, PHYS_RMHD_TM, PRED_MH, RK_LIN, RS_HLL>(c, nb, a, s);                              \
        }                                                                                                        \
        if (c.pred == PRED_MH) {                                                                                 \
            if (c.rs == RS_HLLD) return sweep_one<D, PHYS_MHD, PRED_MH, RK_LIN, RS_HLLD>(c, nb, a, s);            \
            if (c.rs == RS_RUSANOV) return sweep_one<D, PHYS_MHD, PRED_MH, RK_LIN, RS_RUSANOV>(c, nb, a, s);      \
            if (c.rs == RS_HLLC) return sweep_one<D, PHYS_MHD, PRED_MH, RK_LIN, RS_HLLC>(c, nb, a, s);            \
            if (c.rs == RS_ROE) return sweep_one<D, PHYS_MHD, PRED_MH, RK_LIN, RS_ROE>(c, nb, a, s);              \
            return sweep_one<D, PHYS_MHD, PRED_MH, RK_LIN, RS_HLL>(c, nb, a, s);                                  \
        }                                                                                                        \
        if (c.rk == RK_PPM) {                                                                                    \
            if (c.rs == RS_HLLD) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_PPM, RS_HLLD>(c, nb, a, s);          \
            if (c.rs == RS_RUSANOV) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_PPM, RS_RUSANOV>(c, nb, a, s);    \
            if (c.rs == RS_HLLC) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_PPM, RS_HLLC>(c, nb, a, s);          \
            if (c.rs == RS_ROE) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_PPM, RS_ROE>(c, nb, a, s);            \
            return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_PPM, RS_HLL>(c, nb, a, s);                                \
        }                                                                                                        \
        if (c.rk == RK_WENO) {                                                                                   \
            if (c.rs == RS_HLLD) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_WENO, RS_HLLD>(c, nb, a, s);         \
            if (c.rs == RS_RUSANOV) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_WENO, RS_RUSANOV>(c, nb, a, s);   \
            if (c.rs == RS_HLLC) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_WENO, RS_HLLC>(c, nb, a, s);         \
            if (c.rs == RS_ROE) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_WENO, RS_ROE>(c, nb, a, s);           \
            return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_WENO, RS_HLL>(c, nb, a, s);                               \
        }                                                                                                        \
        if (c.rs == RS_HLLD) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_LIN, RS_HLLD>(c, nb, a, s);              \
        if (c.rs == RS_RUSANOV) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_LIN, RS_RUSANOV>(c, nb, a, s);        \
        if (c.rs == RS_HLLC) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_LIN, RS_HLLC>(c, nb, a, s);              \
        if (c.rs == RS_ROE) return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_LIN, RS_ROE>(c, nb, a, s);                \
        return sweep_one<D, PHYS_MHD, PRED_CHAR, RK_LIN, RS_HLL>(c, nb, a, s);                                    \
    }                                                                                                            \
    hipError_t launch_sweep_##SUFFIX(int D, const Combo &c, int nb, const SweepArgs<R> &a, hipStream_t s)      \
    {                                                                                                            \
        if (nb <= 0) return hipSuccess;                                                                          \
        if (D == 0) return sweep_dir<0>(c, nb, a, s);                                                            \
        if (D == 1) return sweep_dir<1>(c, nb, a, s);                                                            \
        return sweep_dir<2>(c, nb, a, s);                                                                        \
    }                                                                                                            \
    /* MHD t^n kernel: the fixed-option variants wherever the option set is   \
       the fast or the par one (the kernel reads GLM and hyperbolic_off only) */ \
    template <int DIM, int RS, int PAR>                                                                          \
    static void tc_mhd(const Combo &c, int nb, const TArgs<R> &a, hipStream_t s)                                \
    {                                                                                                            \
        if (c.fast || c.par) {                                                                                   \
            if constexpr (PAR)                                                                                   \
                hipLaunchKernelGGL((k_tcouple<DIM, PHYS_MHD, RS, 1, VAR_PAR, R>), dim3(nb), dim3(NT), 0, s, a);  \
            else                                                                                                 \
                hipLaunchKernelGGL((k_tcouple<DIM, PHYS_MHD, RS, 0, VAR_FAST, R>), dim3(nb), dim3(NT), 0, s, a); \
        } else {                                                                                                 \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_MHD, RS, PAR, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        }                                                                                                        \
    }                                                                                                            \
    template <int DIM, int PAR>                                                                                  \
    static hipError_t tc_one(const Combo &c, int nb, const TArgs<R> &a, hipStream_t s)                          \
    {                                                                                                            \
        /* the HLL fallback changes only HLLD runs */                                                           \
        if (c.phys == PHYS_RMHD && c.rs == RS_RUSANOV)                                                           \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD, RS_RUSANOV, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.phys == PHYS_RMHD && c.rs == RS_HLLC)                                                         \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD, RS_HLLC, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.phys == PHYS_RMHD && c.rs == RS_HLLD)                                                         \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD, RS_HLLD, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.phys == PHYS_RMHD)                                                                            \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD, RS_HLL, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.phys == PHYS_RMHD_TM && c.rs == RS_RUSANOV)                                                   \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD_TM, RS_RUSANOV, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.phys == PHYS_RMHD_TM && c.rs == RS_HLLC)                                                      \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD_TM, RS_HLLC, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.phys == PHYS_RMHD_TM && c.rs == RS_HLLD)                                                      \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD_TM, RS_HLLD, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.phys == PHYS_RMHD_TM)                                                                         \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_RMHD_TM, RS_HLL, 0, VAR_GENERIC, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.rs == RS_HLLD && a.flag)                                                                      \
            hipLaunchKernelGGL((k_tcouple<DIM, PHYS_MHD, RS_HLLD, PAR, VAR_SHOCK, R>), dim3(nb), dim3(NT), 0, s, a); \
        else if (c.rs == RS_RUSANOV)                                                                             \
            tc_mhd<DIM, RS_RUSANOV, PAR>(c, nb, a, s);                                                           \
        else if (c.rs == RS_HLLC)                                                                                \
            tc_mhd<DIM, RS_HLLC, PAR>(c, nb, a, s);                                                              \
        else if (c.rs == RS_ROE)                                                                                 \
            tc_mhd<DIM, RS_ROE, PAR>(c, nb, a, s);                                                               \
        else if (c.rs == RS_HLLD)                                                                                \
            tc_mhd<DIM, RS_HLLD, PAR>(c, nb, a, s);                                                              \
        else                                                                                                     \
            tc_mhd<DIM, RS_HLL, PAR>(c, nb, a, s);                                                               \
        return hipGetLastError();                                                                                \
    }                                                                                                            \
    hipError_t launch_tcouple_##SUFFIX(int dim, int par, const Combo &c, int nb, const TArgs<R> &a,            \
                                       hipStream_t s)                                                            \
    {                                                                                                            \
        if (nb <= 0) return hipSuccess;                                                                          \
        if (dim == 2) return par ? tc_one<2, 1>(c, nb, a, s) : tc_one<2, 0>(c, nb, a, s);                        \
        return par ? tc_one<3, 1>(c, nb, a, s) : tc_one<3, 0>(c, nb, a, s);                                      \
    }                                                                                                            \
    hipError_t launch_pflux_##SUFFIX(int dim, int div, int nb, const PArgs<R> &a, hipStream_t s)                \
    {                                                                                                            \
        if (nb <= 0) return hipSuccess;                                                                          \
        if (dim == 2 && div) hipLaunchKernelGGL((k_pdiv<2, R>), dim3(nb), dim3(NT), 0, s, a);                    \
        else if (dim == 2) hipLaunchKernelGGL((k_pflux<2, R>), dim3(nb), dim3(NT), 0, s, a);                     \
        else if (div) hipLaunchKernelGGL((k_pdiv<3, R>), dim3(nb), dim3(NT), 0, s, a);                           \
        else hipLaunchKernelGGL((k_pflux<3, R>), dim3(nb), dim3(NT), 0, s, a);                                   \
        return hipGetLastError();                                                                                \
    }                                                                                                            \
    }

// Body of one precision's MT predictor-flux translation unit: k_mtflux for
// every supported (physics, predictor, reconstruction, solver) set.
#define CTU_DEFINE_MT_DISPATCH(R, SUFFIX)                                                                         \
    namespace ctu {                                                                                              \
    template <int D, int PHYS, int PRED, int RK, int RS>                                                         \
    static hipError_t mt_one(int nb, const MtArgs<R> &a, hipStream_t s)                                         \
    {                                                                                                            \
        hipLaunchKernelGGL((k_mtflux<D, PHYS, PRED, RK, RS, R>), dim3(nb), dim3(NT), 0, s, a);                 \
        return hipGetLastError();                                                                                \
    }                                                                                                            \
    template <int D, int PHYS, int PRED, int RK>                                                                 \
    static hipError_t mt_rs(const Combo &c, int nb, const MtArgs<R> &a, hipStream_t s)                          \
    {                                                                                                            \
        if (c.rs == RS_HLLD) return mt_one<D, PHYS, PRED, RK, RS_HLLD>(nb, a, s);                               \
        if constexpr (PHYS == PHYS_MHD) {                                                                        \
            if (c.rs == RS_ROE) return mt_one<D, PHYS, PRED, RK, RS_ROE>(nb, a, s);                             \
        }                                                                                                        \
        if (c.rs == RS_RUSANOV) return mt_one<D, PHYS, PRED, RK, RS_RUSANOV>(nb, a, s);                         \
        if (c.rs == RS_HLLC) return mt_one<D, PHYS, PRED, RK, RS_HLLC>(nb, a, s);                               \
        return mt_one<D, PHYS, PRED, RK, RS_HLL>(nb, a, s);                                                      \
    }                                                                                                            \
    template <int D>                                                                                             \
    static hipError_t mt_dir(const Combo &c, int nb, const MtArgs<R> &a, hipStream_t s)                         \
    {                                                                                                            \
        if (c.phys == PHYS_RMHD) return mt_rs<D, PHYS_RMHD, PRED_MH, RK_LIN>(c, nb, a, s);                      \
        if (c.phys == PHYS_RMHD_TM) return mt_rs<D, PHYS_RMHD_TM, PRED_MH, RK_LIN>(c, nb, a, s);                \
        if (c.pred == PRED_MH) return mt_rs<D, PHYS_MHD, PRED_MH, RK_LIN>(c, nb, a, s);                         \
        if (c.rk == RK_PPM) return mt_rs<D, PHYS_MHD, PRED_CHAR, RK_PPM>(c, nb, a, s);                          \
        if (c.rk == RK_WENO) return mt_rs<D, PHYS_MHD, PRED_CHAR, RK_WENO>(c, nb, a, s);                        \
        return mt_rs<D, PHYS_MHD, PRED_CHAR, RK_LIN>(c, nb, a, s);                                               \
    }                                                                                                            \
    hipError_t launch_mtflux_##SUFFIX(int D, const Combo &c, int nb, const MtArgs<R> &a, hipStream_t s)        \
    {                                                                                                            \
        if (nb <= 0) return hipSuccess;                                                                          \
        if (D == 0) return mt_dir<0>(c, nb, a, s);                                                               \
        if (D == 1) return mt_dir<1>(c, nb, a, s);                                                               \
        return mt_dir<2>(c, nb, a, s);                                                                           \
    }                                                                                                            \
    }
