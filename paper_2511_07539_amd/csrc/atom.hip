// Atom upload, Eq. A2 line optical depths and photoexcitation rates, plus the
// handle and error-string entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "atom.hpp"
#include "common.hpp"

using namespace extrass;

// ---------------------------------------------------------------- handle
extern "C" int extrass_create(extrass_handle* out, int device) {
  if (!out) return EXTRASS_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return EXTRASS_EHIP;
  auto* h = new extrass_ctx();
  h->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete h;
    return EXTRASS_EHIP;
  }
  h->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  // the allocation-free transport's scratch on this device
  if (hipSetDevice(device) != hipSuccess || noalloc_init(device) != hipSuccess) {
    delete h;
    return EXTRASS_EHIP;
  }
  *out = h;
  return EXTRASS_OK;
}

extern "C" int extrass_destroy(extrass_handle h) {
  delete h;
  return EXTRASS_OK;
}

extern "C" const char* extrass_error_string(int code) {
  switch (code) {
    case EXTRASS_OK: return "ok";
    case EXTRASS_EINVAL: return "invalid argument";
    case EXTRASS_ENOSPACE: return "workspace too small";
    case EXTRASS_EHIP: return "HIP runtime error";
    case EXTRASS_EUNSUPPORTED: return "unsupported size";
    default: return "unknown error";
  }
}

extern "C" const char* extrass_last_error(extrass_handle h) {
  return h ? h->last_error.c_str() : "";
}

// ---------------------------------------------------------------- atom
template <class T>
static hipError_t upload(T** dst, const std::vector<T>& v) {
  size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

extern "C" int extrass_atom_create(extrass_handle h, const extrass_atom_desc* d,
                                   extrass_atom_handle* out) {
  if (!h || !d || !out) return fail(h, EXTRASS_EINVAL, "extrass_atom_create: null argument");
  *out = nullptr;
  const int S = d->n_species, N = d->n_levels, T = d->n_trans;
  if (S <= 0 || N <= 0 || T < 0 || !d->species_offset || !d->level_ion || !d->level_energy ||
      !d->level_g || !d->ion_alpha0 || (T > 0 && (!d->trans_lower || !d->trans_upper ||
                                                  !d->trans_A || !d->trans_lambda ||
                                                  !d->trans_upsilon || !d->trans_line)))
    return fail(h, EXTRASS_EINVAL, "extrass_atom_create: missing arrays");
  if (d->species_offset[0] != 0 || d->species_offset[S] != N)
    return fail(h, EXTRASS_EINVAL, "extrass_atom_create: species_offset must span [0, N]");
  auto* a = new extrass_atom_ctx();
  a->S = S;
  a->N = N;
  a->T = T;
  a->off.assign(d->species_offset, d->species_offset + S + 1);
  int maxNs = 0;
  for (int s = 0; s < S; ++s) {
    int Ns = a->off[s + 1] - a->off[s];
    if (Ns <= 0 || Ns > kMaxLevels) {
      delete a;
      return fail(h, EXTRASS_EUNSUPPORTED, "extrass_atom_create: 1..64 levels per species");
    }
    maxNs = std::max(maxNs, Ns);
  }
  a->maxNs = maxNs;
  // per-level data: stage, energy, g, local index of the next stage's ground,
  // and the share of that ground's recombination flux the level receives
  std::vector<int32_t> lv_ion(N), lv_gnext(N, -1), lv_stage_count(S, 0);
  std::vector<double> lv_E(N), lv_g(N), lv_share(N, 0.0);
  for (int s = 0; s < S; ++s) {
    const int b = a->off[s], e = a->off[s + 1];
    int prev = -1, nst = 0;
    for (int i = b; i < e; ++i) {
      int z = d->level_ion[i];
      if (z < 0 || z > 2 || z < prev || z > prev + 1 || (i == b && z != 0)) {
        delete a;
        return fail(h, EXTRASS_EINVAL, "extrass_atom_create: ion stages must be 0,1,2 in order");
      }
      prev = z;
      nst = z + 1;
    }
    lv_stage_count[s] = nst;
    {
      int count[3] = {0, 0, 0};
      for (int i = b; i < e; ++i) ++count[d->level_ion[i]];
      int lanes = 0;
      for (int z = 0; z < nst; ++z) {
        const int B = count[z] + (z + 1 < nst ? 1 : 0);
        a->maxBlock = std::max(a->maxBlock, B);
        lanes += B;
      }
      a->blockLanes = std::max(a->blockLanes, lanes);
      int st[4] = {0, count[0], count[0] + count[1], count[0] + count[1] + count[2]};
      int packed = 0;
      for (int z = 0; z < nst; ++z)
        for (int i = st[z]; i < st[z + 1]; ++i) {
          const int lo = (i == st[z] && z > 0) ? st[z - 1] : st[z];
          const int hi = z + 1 < nst ? st[z + 1] : (e - b) - 1;
          packed += hi - lo + 1;
        }
      a->maxPacked = std::max(a->maxPacked, packed);
    }
    int ground[3] = {-1, -1, -1};
    double sumg[3] = {0, 0, 0};
    for (int i = b; i < e; ++i) {
      int z = d->level_ion[i];
      if (ground[z] < 0) ground[z] = i - b;
      else sumg[z] += d->level_g[i];
    }
    for (int i = b; i < e; ++i) {
      int z = d->level_ion[i];
      lv_ion[i] = z;
      lv_E[i] = d->level_energy[i];
      lv_g[i] = d->level_g[i];
      if (z + 1 < nst) {
        lv_gnext[i] = ground[z + 1];
        if (sumg[z] == 0.0) lv_share[i] = 1.0;
        else if (i - b == ground[z]) lv_share[i] = 1.0 / 3.0;
        else lv_share[i] = (2.0 / 3.0) * d->level_g[i] / sumg[z];
      }
    }
  }
  // transitions grouped by species, with local level indices
  std::vector<int32_t> order(T);
  for (int t = 0; t < T; ++t) order[t] = t;
  auto species_of = [&](int lvl) {
    return int(std::upper_bound(a->off.begin(), a->off.end(), lvl) - a->off.begin()) - 1;
  };
  std::vector<char> seen_pair;
  for (int t = 0; t < T; ++t) {
    int lo = d->trans_lower[t], up = d->trans_upper[t];
    if (lo < 0 || up >= N || lo >= up || species_of(lo) != species_of(up) ||
        d->level_ion[lo] != d->level_ion[up]) {
      delete a;
      return fail(h, EXTRASS_EINVAL, "extrass_atom_create: bad transition levels");
    }
    if (d->trans_line[t] < 0) {
      delete a;
      return fail(h, EXTRASS_EINVAL, "extrass_atom_create: negative line index");
    }
    a->maxLine = std::max(a->maxLine, (int)d->trans_line[t]);
  }
  a->lam_host.assign(d->trans_lambda, d->trans_lambda + T);
  a->lv_ion_host.assign(d->level_ion, d->level_ion + N);
  a->lv_E_host.assign(d->level_energy, d->level_energy + N);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return species_of(d->trans_lower[x]) < species_of(d->trans_lower[y]);
  });
  a->toff.assign(S + 1, 0);
  std::vector<int32_t> tl(T), tu(T), tg(T), tline(T), tlo_glob(T);
  for (int i = 0; i < T; ++i) {
    int t = order[i];
    int s = species_of(d->trans_lower[t]);
    a->toff[s + 1]++;
    tl[i] = d->trans_lower[t] - a->off[s];
    tu[i] = d->trans_upper[t] - a->off[s];
    tg[i] = t;
  }
  for (int s = 0; s < S; ++s) a->toff[s + 1] += a->toff[s];
  std::vector<double> tpack(6 * (size_t)T);
  std::vector<int32_t> tidx(4 * (size_t)T, 0);
  for (int i = 0; i < T; ++i) {
    const int t = order[i];
    const int lo = d->trans_lower[t], up = d->trans_upper[t];
    const double gl = d->level_g[lo], gu = d->level_g[up], lam = d->trans_lambda[t];
    tpack[6 * i + 0] = d->trans_A[t] * lam * lam * lam / (8.0 * M_PI);
    tpack[6 * i + 1] = d->trans_A[t];
    tpack[6 * i + 2] = gu / gl;
    tpack[6 * i + 3] = gl / gu;
    tpack[6 * i + 4] = 8.629e-6 * d->trans_upsilon[t] / gu;
    tpack[6 * i + 5] = d->level_energy[up] - d->level_energy[lo];
    tidx[4 * i + 0] = tl[i];
    tidx[4 * i + 1] = tu[i];
    tidx[4 * i + 2] = tg[i];
  }
  for (int s = 0; s < S; ++s) {  // at most one transition per level pair
    const int Ns = a->off[s + 1] - a->off[s];
    seen_pair.assign((size_t)Ns * Ns, 0);
    for (int i = a->toff[s]; i < a->toff[s + 1]; ++i) {
      char& f = seen_pair[(size_t)tl[i] * Ns + tu[i]];
      if (f) {
        delete a;
        return fail(h, EXTRASS_EINVAL, "extrass_atom_create: two transitions share a level pair");
      }
      f = 1;
    }
  }
  // transitions in the caller's order, for line_tau / rates
  std::vector<int32_t> olo(T), oup(T), oline(T);
  std::vector<double> oA(T), olam(T);
  for (int t = 0; t < T; ++t) {
    olo[t] = d->trans_lower[t];
    oup[t] = d->trans_upper[t];
    oline[t] = d->trans_line[t];
    oA[t] = d->trans_A[t];
    olam[t] = d->trans_lambda[t];
  }
  std::vector<int32_t> toff32(a->toff.begin(), a->toff.end());
  std::vector<int32_t> off32(a->off.begin(), a->off.end());
  std::vector<double> alpha(d->ion_alpha0, d->ion_alpha0 + 3 * S);
  std::vector<int32_t> nstage(lv_stage_count);
  hipError_t e = hipSetDevice(h->device);
  if (e == hipSuccess) e = upload(&a->d.off, off32);
  if (e == hipSuccess) e = upload(&a->d.toff, toff32);
  if (e == hipSuccess) e = upload(&a->d.nstage, nstage);
  if (e == hipSuccess) e = upload(&a->d.lv_ion, lv_ion);
  if (e == hipSuccess) e = upload(&a->d.lv_gnext, lv_gnext);
  if (e == hipSuccess) e = upload(&a->d.lv_E, lv_E);
  if (e == hipSuccess) e = upload(&a->d.lv_g, lv_g);
  if (e == hipSuccess) e = upload(&a->d.lv_share, lv_share);
  if (e == hipSuccess) e = upload(&a->d.t_pack, tpack);
  if (e == hipSuccess) e = upload(&a->d.t_idx, tidx);
  if (e == hipSuccess) e = upload(&a->d.alpha0, alpha);
  if (e == hipSuccess) e = upload(&a->d.o_lo, olo);
  if (e == hipSuccess) e = upload(&a->d.o_up, oup);
  if (e == hipSuccess) e = upload(&a->d.o_line, oline);
  if (e == hipSuccess) e = upload(&a->d.o_A, oA);
  if (e == hipSuccess) e = upload(&a->d.o_lam, olam);
  {
    std::vector<double> oK(T), orr(T);
    for (int t = 0; t < T; ++t) {
      const double gl = d->level_g[olo[t]], gu = d->level_g[oup[t]], l = olam[t];
      oK[t] = oA[t] / (8.0 * M_PI) * (gu / gl) * l * l * l;
      orr[t] = gl / gu;
    }
    if (e == hipSuccess) e = upload(&a->d.o_K, oK);
    if (e == hipSuccess) e = upload(&a->d.o_r, orr);
  }
  if (e != hipSuccess) {
    extrass_atom_destroy(a);
    return fail(h, EXTRASS_EHIP, std::string("extrass_atom_create: ") + hipGetErrorString(e));
  }
  a->device = h->device;
  *out = a;
  return EXTRASS_OK;
}

extern "C" int extrass_atom_destroy(extrass_atom_handle a) {
  if (!a) return EXTRASS_OK;
  void* ptrs[] = {a->d.off, a->d.toff, a->d.nstage, a->d.lv_ion, a->d.lv_gnext, a->d.lv_E,
                  a->d.lv_g, a->d.lv_share, a->d.t_pack, a->d.t_idx, a->d.alpha0, a->d.o_lo,
                  a->d.o_up, a->d.o_line, a->d.o_A, a->d.o_lam, a->d.o_K, a->d.o_r};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete a;
  return EXTRASS_OK;
}

// ---------------------------------------------------------------- Eq. A2
// A tile of cpt cells per pass: their populations go to LDS, then the
// tile's (cell, transition) entries are formed in order, so the threads'
// writes of both outputs are contiguous across the tile. (One cell per pass
// left the last of its four passes over 800 transitions a quarter busy and
// synchronised the work-group per cell.) With STAGE, the transitions' levels
// and constants are read into LDS once per work-group, which then walks its
// tiles; each thread steps its (cell, transition) position by the block size
// instead of dividing.
template <bool STAGE>
__global__ __launch_bounds__(256) void k_line_tau(int64_t n_cells, int N, int T, int cpt,
                                                 const double* __restrict__ pops,
                                                 const int32_t* __restrict__ lo,
                                                 const int32_t* __restrict__ up,
                                                 const double* __restrict__ K,
                                                 const double* __restrict__ r, double t_exp,
                                                 double* __restrict__ tau,
                                                 double* __restrict__ fcorr) {
  extern __shared__ double smem[];
  double* pc = smem;                                   // [cpt * N] populations of the tile
  double* sK = smem + (size_t)cpt * N;                 // [T] (STAGE)
  double* sR = sK + T;                                 // [T]
  int2* sLU = reinterpret_cast<int2*>(sR + T);         // [T] lower, upper level
  if constexpr (STAGE)
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
      sK[t] = K[t];
      sR[t] = r[t];
      sLU[t] = make_int2(lo[t], up[t]);
    }
  for (int64_t c0 = (int64_t)blockIdx.x * cpt; c0 < n_cells; c0 += (int64_t)gridDim.x * cpt) {
    const int nc = (int)(n_cells - c0 < cpt ? n_cells - c0 : cpt);
    for (int i = threadIdx.x; i < nc * N; i += blockDim.x) pc[i] = pops[c0 * N + i];
    __syncthreads();
    double* tau_t = tau + c0 * T;
    double* fc_t = fcorr + c0 * T;
    int k = 0, t = threadIdx.x;
    while (t >= T) {
      t -= T;
      ++k;
    }
    for (int e = threadIdx.x; e < nc * T; e += blockDim.x) {
      const int2 lu = STAGE ? sLU[t] : make_int2(lo[t], up[t]);
      const double rt = STAGE ? sR[t] : r[t];
      const double Kt = STAGE ? sK[t] : K[t];
      const double nl = pc[k * N + lu.x], nu = pc[k * N + lu.y];
      double tv = 0.0, fc = 1.0;
      if (nl > 0.0) {
        fc = 1.0 - rt * nu / nl;
        tv = Kt * nl * fc * t_exp;
      }
      tau_t[e] = tv;
      fc_t[e] = fc;
      t += blockDim.x;
      while (t >= T) {
        t -= T;
        ++k;
      }
    }
    __syncthreads();
  }
}

extern "C" int extrass_line_tau(extrass_handle h, extrass_atom_handle a, int64_t n_cells,
                                const double* pops, double t_exp, double* tau_ct,
                                double* fcorr_ct, void* stream) {
  if (!h || !a || !pops || !tau_ct || !fcorr_ct || n_cells < 0)
    return fail(h, EXTRASS_EINVAL, "extrass_line_tau: bad argument");
  if (n_cells == 0 || a->T == 0) return EXTRASS_OK;
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  if (a->N > 8192)  // a cell's populations are staged in 64 KB of LDS
    return fail(h, EXTRASS_EUNSUPPORTED, "extrass_line_tau: more than 8192 levels");
  // cells per tile: up to 4, within 64 KB of LDS
  const int cpt = std::max(1, std::min(4, 8192 / a->N));
  const int64_t tiles = (n_cells + cpt - 1) / cpt;
  const size_t pop_bytes = sizeof(double) * a->N * cpt;
  // the transition table (24 B per transition) joins the tile in LDS when
  // both fit in 48 KB; the grid is then what stays resident (each
  // work-group walks many tiles with the table loaded once)
  const size_t stage_bytes = pop_bytes + (size_t)24 * a->T;
  const bool stage = stage_bytes <= 48 * 1024;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (stage) {
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / stage_bytes));
    const int64_t blocks = std::min<int64_t>(tiles, (int64_t)h->num_cus * per_cu);
    hipLaunchKernelGGL(k_line_tau<true>, dim3((unsigned)blocks), dim3(256), stage_bytes, st,
                       n_cells, a->N, a->T, cpt, pops, a->d.o_lo, a->d.o_up, a->d.o_K, a->d.o_r,
                       t_exp, tau_ct, fcorr_ct);
  } else {
    const int64_t blocks = std::min<int64_t>(tiles, (int64_t)h->num_cus * 32);
    hipLaunchKernelGGL(k_line_tau<false>, dim3((unsigned)blocks), dim3(256), pop_bytes, st,
                       n_cells, a->N, a->T, cpt, pops, a->d.o_lo, a->d.o_up, a->d.o_K, a->d.o_r,
                       t_exp, tau_ct, fcorr_ct);
  }
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}

// ---------------------------------------------------------------- rates
__global__ void k_rates(int64_t n_cells, int L, int N, int T, const double* __restrict__ est,
                        const double* __restrict__ pops, const int32_t* __restrict__ lo,
                        const int32_t* __restrict__ line, CellVolume V, double* __restrict__ gamma) {
  const int64_t total = n_cells * T;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / T;
    const int t = static_cast<int>(e - c * T);
    const double Nl = pops[c * N + lo[t]] * V(c);
    const double x = est[c * L + line[t]];
    gamma[e] = Nl > 0.0 ? x / Nl : 0.0;
  }
}

extern "C" int extrass_rates(extrass_handle h, extrass_atom_handle a, const extrass_grid* g,
                             double t_exp, const double* est, const double* pops,
                             double* gamma_pe, void* stream) {
  if (!h || !a || !g || !est || !pops || !gamma_pe || !grid_shape_ok(g) || g->n_lines <= 0 ||
      !(t_exp > 0.0))
    return fail(h, EXTRASS_EINVAL, "extrass_rates: bad argument");
  if (a->maxLine >= g->n_lines)
    return fail(h, EXTRASS_EINVAL, "extrass_rates: a transition's line index is beyond the grid's lines");
  const int64_t n_cells = grid_cell_count(g);
  if (a->T == 0) return EXTRASS_OK;
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  const CellVolume V = grid_volumes(g, t_exp);
  const int64_t total = n_cells * a->T;
  int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_rates, dim3((unsigned)blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), n_cells, (int)g->n_lines, a->N, a->T, est,
                     pops, a->d.o_lo, a->d.o_line, V, gamma_pe);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}
