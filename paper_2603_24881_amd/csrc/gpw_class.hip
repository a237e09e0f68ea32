// Launches of the kernels of one (l_a, l_b) class.  This source is compiled
// once per class, with GPW_CLS set to the class index (ss ps pp ds dp dd fs
// fp fd ff gs gp gd gf gg), so that the templated kernels of the classes compile in
// parallel translation units; launch_class() dispatches to them.
#include "gpw_kernels.h"

#ifndef GPW_CLS
#error "compile with -DGPW_CLS=<class index>"
#endif

namespace gpw {

#define GPW_CAT2(a, b) a##b
#define GPW_CAT(a, b) GPW_CAT2(a, b)
#define GPW_LAUNCH_FN GPW_CAT(launch_class_, GPW_CLS)

template <int LA, int LB, typename T>
static void launch_lists(const ClassLaunch &cl)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    const hipStream_t st = cl.st;
    const size_t smem = cl.smem, smem_t = cl.smem_t;
    // packed coefficients (general cells: Cartesian tensors, then their
    // rewrite on the index offset)
    cl.packs.launch([&](const SegTable<PackSeg> &tb, unsigned g) {
        if constexpr (rho_tensor(LA, LB))
            hipLaunchKernelGGL((k_pack_density<T, LA, LB>), dim3(g), dim3(256), 0, st, tb);
        else
            hipLaunchKernelGGL((k_pack_direct<T, NA, NB>), dim3(g), dim3(256), 0, st, tb);
    }, false);
    cl.packs_t.launch([&](const SegTable<PackSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_pack_density<T, LA, LB>), dim3(g), dim3(256), 0, st, tb);
    }, false);
    cl.tpacks.launch([&](const SegTable<PackSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_pack_tau<T, LA, LB>), dim3(g), dim3(256), 0, st, tb);
    }, false);
    cl.idxs.launch([&](const SegTable<IdxSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_to_index<T>), dim3(g), dim3(256), 0, st, tb);
    }, false);
    using RS = RhoSplit<LA, LB>;
    cl.rhos.launch([&](const SegTable<RhoSeg> &tb, unsigned g) {
        if constexpr (RS::two)
            hipLaunchKernelGGL((k_rho2<LA, LB, RS::wpe2, T>), dim3(g), dim3(128), 0, st, tb);
        else
            hipLaunchKernelGGL((k_rho<LA, LB, RS::npass, RS::wpe, RS::stage, RS::pref, T>), dim3(g), dim3(64), 0, st,
                               tb);
    }, true);
    cl.rhos_t.launch([&](const SegTable<RhoSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_rho_tri<LA, LB, TauSplit<LA + LB>::npass, T>), dim3(g), dim3(64), 0, st, tb);
    }, true);
    cl.mats.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_mat<LA, LB, T>), dim3(g), dim3(64), smem, st, tb);
    }, true);
    cl.mats_t.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_mat<LA, LB, T, true>), dim3(g), dim3(64), smem_t, st, tb);
    }, true);
    cl.grads.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_grad<LA, LB, T>), dim3(g), dim3(64), smem, st, tb);
    }, true);
    cl.grads_t.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_grad<LA, LB, T, true>), dim3(g), dim3(64), smem_t, st, tb);
    }, true);
    using TS = TauSplit<LA + LB + 2>;
    cl.taus.launch([&](const SegTable<RhoSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_tau<LA, LB, TS::npass, TS::wpe, T>), dim3(g), dim3(64), 0, st, tb);
    }, true);
    cl.taus_t.launch([&](const SegTable<RhoSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_tau_tri<LA, LB, TS::npass, T>), dim3(g), dim3(64), 0, st, tb);
    }, true);
    cl.mtaus.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_mat_tau<LA, LB, T>), dim3(g), dim3(64), smem, st, tb);
    }, true);
    cl.mtaus_t.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_mat_tau<LA, LB, T, true>), dim3(g), dim3(64), smem_t, st, tb);
    }, true);
    cl.gtaus.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_grad_tau<LA, LB, T>), dim3(g), dim3(64), smem, st, tb);
    }, true);
    cl.gtaus_t.launch([&](const SegTable<PairSeg> &tb, unsigned g) {
        hipLaunchKernelGGL((k_grad_tau<LA, LB, T, true>), dim3(g), dim3(64), smem_t, st, tb);
    }, true);
}

void GPW_LAUNCH_FN(const ClassLaunch &cl)
{
    constexpr int LA = cls_la_c(GPW_CLS), LB = cls_lb_c(GPW_CLS);
    if (cl.fp32)
        launch_lists<LA, LB, float>(cl);
    else
        launch_lists<LA, LB, double>(cl);
}

}  // namespace gpw
