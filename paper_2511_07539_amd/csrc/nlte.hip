// Host entry of the NLTE solve and the status initialisation; the solver
// kernels are in nlte_kernel.hpp, instantiated in nlte_blocks.hip and
// nlte_whole.hip.
#include "nlte_kernel.hpp"

namespace extrass {
namespace {

__global__ void k_nlte_init(int64_t C, int S, const double* n_species, int32_t* status,
                            int32_t* iters, unsigned long long* queue) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    bool empty = true;
    for (int s = 0; s < S; ++s)
      if (n_species[c * S + s] > 0.0) empty = false;
    status[c] = empty ? 3 : 0;
    if (iters) iters[c] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0ull;
}

}  // namespace
}  // namespace extrass

using namespace extrass;

extern "C" size_t extrass_nlte_workspace(extrass_atom_handle a, int64_t n_cells) {
  (void)a;
  (void)n_cells;
  return 512;
}

extern "C" int extrass_nlte_solve(extrass_handle h, extrass_atom_handle a, const extrass_cells* cl,
                                  const extrass_nlte_opts* o, double* pops, int32_t* status,
                                  int32_t* iters, void* ws, size_t ws_bytes, void* stream) {
  if (!h || !a || !cl || !o || !pops || !status || !ws)
    return fail(h, EXTRASS_EINVAL, "extrass_nlte_solve: null argument");
  if (cl->n_cells < 0 || !cl->T_e || !cl->n_e || !cl->n_species || !cl->gamma_ion ||
      o->max_iter < 0 || !(o->tol > 0.0))
    return fail(h, EXTRASS_EINVAL, "extrass_nlte_solve: bad cells or options");
  if (ws_bytes < extrass_nlte_workspace(a, cl->n_cells))
    return fail(h, EXTRASS_ENOSPACE, "extrass_nlte_solve: workspace too small");
  if (cl->n_cells == 0) return EXTRASS_OK;
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* queue = static_cast<unsigned long long*>(ws);
  {
    int64_t blocks = std::min<int64_t>((cl->n_cells + 255) / 256, 4096);
    hipLaunchKernelGGL(k_nlte_init, dim3((unsigned)blocks), dim3(256), 0, st, cl->n_cells, a->S,
                       cl->n_species, status, iters, queue);
  }
  NArgs A{};
  A.S = a->S;
  A.N = a->N;
  A.T = a->T;
  A.C = cl->n_cells;
  A.t_exp = cl->t_exp;
  A.off = a->d.off;
  A.toff = a->d.toff;
  A.nstage = a->d.nstage;
  A.lv_ion = a->d.lv_ion;
  A.lv_gnext = a->d.lv_gnext;
  A.lv_E = a->d.lv_E;
  A.lv_g = a->d.lv_g;
  A.lv_share = a->d.lv_share;
  A.t_pack = a->d.t_pack;
  A.t_idx = a->d.t_idx;
  A.alpha0 = a->d.alpha0;
  A.T_e = cl->T_e;
  A.n_e = cl->n_e;
  A.n_species = cl->n_species;
  A.gamma_ion = cl->gamma_ion;
  A.gamma_pe = cl->gamma_pe;
  A.gamma_pi = cl->gamma_pi;
  A.max_iter = o->max_iter;
  A.tol = o->tol;
  A.use_guess = o->use_guess;
  A.warm_budget = o->warm_budget;
  A.pops = pops;
  A.status = status;
  A.iters = iters;
  A.queue = queue;
  A.NP = a->maxNs | 1;
  A.gsz = a->maxNs * A.NP;
  A.block_rows = (a->blockLanes + 1) & ~1;
  const bool blocks_fit = a->maxBlock <= 32 && a->blockLanes <= 64;
  if (o->factor_fp32 && !blocks_fit)
    return fail(h, EXTRASS_EUNSUPPORTED,
                "extrass_nlte_solve: the mixed-precision pass needs stage blocks of at most 32 states "
                "in 64 lanes");
  // stage blocks: kernels for blocks of at most 12, 16, 21, 22, 24 or 32
  // states (the reduction runs NTB - 1 unrolled steps on NTB-entry register
  // rows, so a bound one above the largest block costs a step and an entry:
  // 21 is the 20/15/15 atom's largest block)
  const int ntb = a->maxBlock <= 12 ? 12
                : a->maxBlock <= 16 ? 16
                : a->maxBlock <= 21 ? 21
                : a->maxBlock <= 22 ? 22
                : a->maxBlock <= 24 ? 24 : 32;
  // whole system: kernels for species of at most 16, 24, 32, 40, 50 or 64 levels
  const int nt = a->maxNs <= 16 ? 16
               : a->maxNs <= 24 ? 24
               : a->maxNs <= 32 ? 32
               : a->maxNs <= 40 ? 40
               : a->maxNs <= 50 ? 50 : 64;
  const size_t lds = sizeof(double) *
                     (192 + (blocks_fit ? std::max<size_t>(block_scratch(ntb, A.block_rows),
                                                           (size_t)a->maxPacked)
                                        : (size_t)A.gsz + 64));
  const int64_t items = cl->n_cells * a->S;
  int per_cu = (int)std::min<size_t>(16, (160 * 1024) / std::max<size_t>(lds, 1));
  if (per_cu < 1) per_cu = 1;
  int64_t blocks = std::min<int64_t>((int64_t)h->num_cus * per_cu, items);
  if (blocks < 1) blocks = 1;
  // The stage-block reduction serves atoms whose blocks fit (at most 32
  // states each, side by side in 64 lanes), in FP64 or with the fixed-point
  // steps in FP32; otherwise the whole-system register reduction
  // (FP64), compiled for a few system sizes, the smallest that holds the
  // largest species.
  const bool launched =
      blocks_fit ? (o->factor_fp32 ? launch_nlte_blocks_mixed(ntb, (unsigned)blocks, lds, st, A)
                                   : launch_nlte_blocks(ntb, (unsigned)blocks, lds, st, A))
                 : launch_nlte_whole(nt, (unsigned)blocks, lds, st, A);
  if (!launched) return fail(h, EXTRASS_EINVAL, "extrass_nlte_solve: no kernel for this atom");
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}
