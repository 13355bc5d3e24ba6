// bttb_cols.hip -- dispatch of the column kernels of the two products
// (cols_impl.h) on the transform length; the kernels of each length are
// instantiated in bttb_cols_*.hip, one group of lengths per translation
// unit so that they compile in parallel.
#include "kern_common.h"

namespace bttbk {

// defined in cols_impl.h, instantiated per length in bttb_cols_*.hip
template <typename T, int ACC, int NN>
hipError_t cols_fwd_n(int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s);
template <typename T, int NN>
hipError_t cols_fin_n(int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s);
template <typename T, int NN>
hipError_t cols_tr_n(int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s);

template <typename T, int ACC>
hipError_t launch_cols_fwd(int N, int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_FWD(NN) return cols_fwd_n<T, ACC, NN>(tile, form, jobs, tw, s)
    BTTB_LEN_SWITCH(N, L_FWD)
#undef L_FWD
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_cols_fwd_fin(int N, int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_FIN(NN) return cols_fin_n<T, NN>(tile, form, jobs, tw, s)
    BTTB_LEN_SWITCH(N, L_FIN)
#undef L_FIN
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_cols_tr(int N, int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_TR(NN) return cols_tr_n<T, NN>(tile, form, jobs, tw, s)
    BTTB_LEN_SWITCH(N, L_TR)
#undef L_TR
    return hipErrorInvalidValue;
}

template hipError_t launch_cols_fwd<double, ACC_PLAIN>(int, int, int, const ColJobs&, const double2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_PLAIN>(int, int, int, const ColJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_TWOSUM>(int, int, int, const ColJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_WIDE>(int, int, int, const ColJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_fwd_fin<double>(int, int, int, const ColJobs&, const double2*, hipStream_t);
template hipError_t launch_cols_fwd_fin<float>(int, int, int, const ColJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_tr<double>(int, int, int, const ColJobs&, const double2*, hipStream_t);
template hipError_t launch_cols_tr<float>(int, int, int, const ColJobs&, const float2*, hipStream_t);

}  // namespace bttbk
