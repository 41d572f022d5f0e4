// Many independent networks (uneven widths and N) in one call: exact H and/or OPG of
// every network, FP32.  The per-example passes and curvature factors of each network
// run as small launches (FP64 scratch shared between networks, results cast to FP32
// into per-network regions); then every P x P tile of every network goes through one
// persistent launch that hands out tiles from a global counter (a second persistent
// launch adds the cross-layer term of H, which accumulates onto the first).
#include <algorithm>
#include <cstring>
#include <vector>

#include "api_internal.h"
#include "mfma.h"

namespace hs {

namespace {

struct BNet {
  Model m;
  int64_t N = 0;
  OpgBufs<float> ops;                        // abar, delta in FP32 (persistent)
  std::vector<std::vector<float*>> G, K;     // [mm][l] FP32 factors (persistent)
  std::vector<float*> D1;                    // [mm] sigma'^(mm) transposed, FP32
};

struct BPlan {
  std::vector<BNet> nets;
  size_t scratch_bytes = 0;
  KrgJob* jobs = nullptr;
  unsigned long long* counter = nullptr;
  int* flags = nullptr;
  int64_t njobs_max = 0;
  float* pdws = nullptr;  // pair-diagonal blocks as one product (one network at a time)
};

// FP64 scratch needed by one network: per-example caches plus the factors of one column layer.
size_t scratch_of(const Model& m, int64_t N) {
  Arena ar(nullptr);
  Prep p;
  plan_prep(ar, m, N, p, true);
  const size_t base = ar.used;
  size_t peak = base;
  for (int mm = 2; mm <= m.L; ++mm) {
    Arena a2(nullptr);
    a2.used = base;
    const int64_t Tm = m.T[mm - 1];
    for (int l = mm + 1; l <= m.L; ++l) a2.take<double>(m.T[l - 1] * Tm * N);
    for (int l = mm + 1; l <= m.L - 1; ++l) a2.take<double>(m.T[l - 1] * Tm * N);
    for (int l = mm; l <= m.L; ++l) a2.take<double>(m.T[l - 1] * Tm * N);
    peak = std::max(peak, a2.used);
  }
  return peak;
}

int64_t jobs_of(const Model& m) {
  const int64_t Lm = m.L - 1;  // weight layers
  return 2 * Lm * (Lm + 1) / 2 + Lm * (Lm - 1) / 2 + 1;
}

size_t plan_batched(Arena& ar, int64_t M, const hess_mlp* models, const hess_data* datas, BPlan& bp,
                    hess_ctx* ctx, bool need_ptrs, hess_status* st) {
  bp.nets.assign(M, BNet());
  size_t scratch = 0;
  int64_t nj = 0;
  for (int64_t i = 0; i < M; ++i) {
    BNet& b = bp.nets[i];
    if ((*st = validate_mlp(ctx, &models[i], b.m, need_ptrs)) != HESS_OK) return 0;
    if ((*st = validate_data(ctx, &datas[i], need_ptrs)) != HESS_OK) return 0;
    b.N = datas[i].N;
    scratch = std::max(scratch, scratch_of(b.m, b.N));
    nj += jobs_of(b.m);
  }
  bp.scratch_bytes = scratch;
  (void)ar.take<char>(scratch);  // scratch at offset 0
  bp.flags = ar.take<int>(2 * M);
  bp.counter = ar.take<unsigned long long>(8);
  bp.njobs_max = nj;
  bp.jobs = ar.take<KrgJob>(nj);
  int64_t pf = 0;
  for (int64_t i = 0; i < M; ++i)
    for (int mm = 2; mm <= bp.nets[i].m.L - 1; ++mm) {
      const int64_t f = pairdiag_block_floats(bp.nets[i].m, bp.nets[i].N, mm);
      if (f * 4 <= kPairdiagMaxBytes) pf = std::max(pf, f);
    }
  if (pf > 0) bp.pdws = ar.take<float>((size_t)pf);
  for (int64_t i = 0; i < M; ++i) {
    BNet& b = bp.nets[i];
    const Model& m = b.m;
    const int L = m.L;
    const int64_t N = b.N;
    // the operand layout needs lda, which plan_prep fixes
    Arena probe(nullptr);
    Prep p;
    plan_prep(probe, m, N, p, true);
    plan_opg_ops<float>(ar, m, N, p, b.ops);
    b.G.assign(L + 1, std::vector<float*>(L + 1, nullptr));
    b.K.assign(L + 1, std::vector<float*>(L + 1, nullptr));
    b.D1.assign(L + 1, nullptr);
    for (int mm = 2; mm <= L; ++mm) {
      const int64_t Tm = m.T[mm - 1];
      for (int l = mm; l <= L; ++l) b.G[mm][l] = ar.take<float>(m.T[l - 1] * Tm * N);
      for (int l = mm + 1; l <= L - 1; ++l) b.K[mm][l] = ar.take<float>(m.T[l - 1] * Tm * N);
      if (mm < L) b.D1[mm] = ar.take<float>(Tm * N);
    }
  }
  *st = HESS_OK;
  return ar.used;
}

}  // namespace

hess_status batched_workspace(hess_ctx* ctx, int64_t M, const hess_mlp* models, const hess_data* datas,
                              size_t* bytes) {
  if (M < 1 || !models || !datas) return fail(ctx, HESS_E_ARG, "batched: M >= 1 models and data required");
  Arena ar(nullptr);
  BPlan bp;
  hess_status st = HESS_OK;
  *bytes = plan_batched(ar, M, models, datas, bp, ctx, false, &st);
  return st;
}

}  // namespace hs

using namespace hs;

extern "C" hess_status hess_batched(hess_ctx* ctx, int64_t M, const hess_mlp* models, const hess_data* datas,
                                    int prec, void* const* H, void* const* G, void* ws, size_t ws_bytes) {
  Exec ex;
  hess_status st = begin(ctx, ex);
  if (st != HESS_OK) return st;
  if (prec != HESS_P_F32 && prec != HESS_P_F32_SPLIT)
    return fail(ctx, HESS_E_UNSUPPORTED, "batched: HESS_P_F32 or HESS_P_F32_SPLIT");
  ex.split = prec == HESS_P_F32_SPLIT;
  if (M < 1 || !models || !datas || (!H && !G)) return fail(ctx, HESS_E_ARG, "batched: bad arguments");
  Arena probe(nullptr);
  BPlan bp0;
  const size_t need = plan_batched(probe, M, models, datas, bp0, ctx, true, &st);
  if (st != HESS_OK) return st;
  size_t out_bytes = 0;
  for (int64_t i = 0; i < M; ++i)
    out_bytes += (size_t)bp0.nets[i].m.P * bp0.nets[i].m.P * 4 * ((H && H[i] ? 1 : 0) + (G && G[i] ? 1 : 0));
  if ((st = check_ws(ctx, need, ws, ws_bytes, out_bytes)) != HESS_OK) return st;
  Arena ar(ws);
  BPlan bp;
  plan_batched(ar, M, models, datas, bp, ctx, true, &st);
  void* scratch = ws;

  // input checks for every network, one read-back
  if (ctx->check_inputs) {
    hipMemsetAsync(bp.flags, 0, 2 * M * sizeof(int), ex.stream);
    for (int64_t i = 0; i < M; ++i) {
      const Model& m = bp.nets[i].m;
      for (int k = 0; k < m.L - 1; ++k) {
        check_finite(ex, m.W[k], m.dtype, m.T[k + 1] * m.T[k], bp.flags + 2 * i);
        check_finite(ex, m.b[k], m.dtype, m.T[k + 1], bp.flags + 2 * i);
      }
      check_finite(ex, datas[i].X, datas[i].dtype, datas[i].N * m.T[0], bp.flags + 2 * i);
      check_onehot(ex, datas[i].Y, datas[i].dtype, datas[i].N, m.T[m.L - 1], bp.flags + 2 * i + 1);
    }
    std::vector<int> h(2 * M, 0);
    hipMemcpyAsync(h.data(), bp.flags, 2 * M * sizeof(int), hipMemcpyDeviceToHost, ex.stream);
    if (hipStreamSynchronize(ex.stream) != hipSuccess) return fail(ctx, HESS_E_DEVICE, "batched: input check");
    if (ctx->fault_hit) return fail(ctx, HESS_E_DEVICE, "injected device fault");
    for (int64_t i = 0; i < M; ++i) {
      if (h[2 * i]) return fail(ctx, HESS_E_NONFINITE, "network " + std::to_string(i) + ": non-finite input");
      if (h[2 * i + 1]) return fail(ctx, HESS_E_LABEL, "network " + std::to_string(i) + ": Y not one-hot");
    }
  }

  // per-network passes and FP32 factors; tile jobs, grouped by units-per-tile bound
  // (2, 5, 9): one persistent launch per phase and bound, so that every launch reserves
  // only the LDS its tiles need
  constexpr int NU = 3;
  auto ugrp = [](int maxu) { return maxu == 2 ? 0 : (maxu == 5 ? 1 : 2); };
  std::vector<KrgJob> jobsA[NU], jobsB[NU];
  double flopsA[NU] = {0, 0, 0}, flopsB[NU] = {0, 0, 0};
  std::vector<KrgArgs<float, float>> missA, missB;  // contractions too large for the persistent launch
  std::vector<KrgArgs<float, float>> pdiag;         // pair-diagonal blocks done as one product
  auto add = [&](bool phaseA, const KrgArgs<float, float>& a) {
    if (!krg_persistent_fits(a)) {
      (phaseA ? missA : missB).push_back(a);
      return;
    }
    const int g = ugrp(krg_persistent_maxu(a));
    std::vector<KrgJob>& v = phaseA ? jobsA[g] : jobsB[g];
    KrgJob j;
    j.a = a;
    j.mode = a.wmode;
    int64_t tc = 0;
    const int64_t nt = krg_tiles(a, &tc);
    j.tiles_c = tc;
    j.first = v.empty() ? 0 : v.back().first + krg_tiles(v.back().a, &tc);
    if (nt > 0) v.push_back(j);
    const double Pr = (double)a.r.n_units * a.r.len, Pc = (double)a.c.n_units * a.c.len;
    double e = a.symmetric ? Pr * (Pr + 1) / 2 : Pr * Pc;
    if (a.wmode == KRG_PAIR_DIAG) e = (double)std::min(a.r.n_units, a.c.n_units) * a.r.len * a.c.len;
    (phaseA ? flopsA : flopsB)[g] += 2.0 * a.N * e;
  };
  for (int64_t i = 0; i < M; ++i) {
    BNet& b = bp.nets[i];
    const Model& m = b.m;
    const int L = m.L;
    const int64_t N = b.N;
    Arena sa(scratch);
    Prep p;
    plan_prep(sa, m, N, p, true);
    const size_t base = sa.used;
    run_prep(ex, m, &datas[i], p, true);
    cast_ops<float>(ex, m, p, b.ops);
    float* Hi = (H && H[i]) ? static_cast<float*>(H[i]) : nullptr;
    float* Gi = (G && G[i]) ? static_cast<float*>(G[i]) : nullptr;
    for (int mm = 2; mm <= L && Hi; ++mm) {
      const int64_t Tm = m.T[mm - 1];
      Arena a2(scratch);
      a2.used = base;
      HFactors f;
      f.F.assign(L + 1, nullptr);
      f.K.assign(L + 1, nullptr);
      f.G.assign(L + 1, nullptr);
      for (int l = mm + 1; l <= L; ++l) f.F[l] = a2.take<double>(m.T[l - 1] * Tm * N);
      for (int l = mm + 1; l <= L - 1; ++l) f.K[l] = a2.take<double>(m.T[l - 1] * Tm * N);
      for (int l = mm; l <= L; ++l) f.G[l] = a2.take<double>(m.T[l - 1] * Tm * N);
      compute_factors(ex, m, N, 0, p, f, mm);
      for (int l = mm; l <= L; ++l) cast_copy<float>(ex, f.G[l], b.G[mm][l], m.T[l - 1] * Tm * N);
      for (int l = mm + 1; l <= L - 1; ++l) cast_copy<float>(ex, f.K[l], b.K[mm][l], m.T[l - 1] * Tm * N);
      if (mm < L) cast_copy<float>(ex, p.D1T[mm], b.D1[mm], Tm * N);
    }
    const double invN = 1.0 / (double)N;
    for (int l = 2; l <= L; ++l)
      for (int mm = 2; mm <= l; ++mm) {
        KrgArgs<float, float> a;
        a.r = side_layer<float>(m, l, b.ops.abar[l - 1], p.lda[l - 1], nullptr, 0);
        a.c = side_layer<float>(m, mm, b.ops.abar[mm - 1], p.lda[mm - 1], nullptr, 0);
        a.ldo = m.P;
        a.symmetric = l == mm;
        a.accumulate = 0;
        a.mirror = 1;
        a.scale = invN;
        a.N = N;
        if (Gi) {
          KrgArgs<float, float> g = a;
          g.r.scale = b.ops.delta[l];
          g.r.ld_scale = m.T[l - 1];
          g.c.scale = b.ops.delta[mm];
          g.c.ld_scale = m.T[mm - 1];
          g.wmode = KRG_RANK1;
          g.wts = nullptr;
          g.ldw = 0;
          g.out = Gi;
          add(true, g);
        }
        if (Hi) {
          KrgArgs<float, float> h = a;
          h.wmode = KRG_PAIR_FULL;
          h.wts = b.G[mm][l];
          h.ldw = N;
          h.out = Hi;
          add(true, h);
          if (l > mm) {
            KrgArgs<float, float> t2 = h;
            KrgSide<float> r;
            r.src = b.ops.delta[l];
            r.ld = m.T[l - 1];
            r.n_units = (int32_t)m.T[l - 2];
            r.len = (int32_t)m.T[l - 1];
            r.pad = (int32_t)rup(r.len, 16);
            r.scale = nullptr;
            r.ld_scale = 0;
            r.perm = 1;
            r.off = m.offW[l - 2];
            r.Tin = (int32_t)m.T[l - 2];
            r.Tout = (int32_t)m.T[l - 1];
            t2.r = r;
            t2.symmetric = 0;
            t2.accumulate = 1;
            if (l - 1 == mm) {
              t2.wmode = KRG_PAIR_DIAG;
              t2.wts = b.D1[mm];
              if (bp.pdws && pairdiag_block_floats(m, N, mm) * 4 <= kPairdiagMaxBytes) {
                pdiag.push_back(t2);  // as hess_exact does it
                continue;
              }
            } else {
              t2.wmode = KRG_PAIR_FULL;
              t2.wts = b.K[mm][l - 1];
            }
            add(false, t2);
          }
        }
      }
  }
  // upload the job lists and run the persistent launches (phase A, then B)
  const int u_of[NU] = {2, 5, 9};
  std::vector<KrgJob> all;
  int64_t offA[NU], offB[NU];
  for (int g = 0; g < NU; ++g) {
    offA[g] = (int64_t)all.size();
    all.insert(all.end(), jobsA[g].begin(), jobsA[g].end());
  }
  for (int g = 0; g < NU; ++g) {
    offB[g] = (int64_t)all.size();
    all.insert(all.end(), jobsB[g].begin(), jobsB[g].end());
  }
  if (!all.empty())
    hipMemcpyAsync(bp.jobs, all.data(), all.size() * sizeof(KrgJob), hipMemcpyHostToDevice, ex.stream);
  auto total_of = [](const std::vector<KrgJob>& v) {
    int64_t tc = 0;
    return v.empty() ? (int64_t)0 : v.back().first + krg_tiles(v.back().a, &tc);
  };
  // Phase A writes its blocks (no accumulation), so its configuration may be tuned: probes
  // on the first two device rounds of tiles write outputs that the full launch overwrites.
  // Every FP32 configuration gives the same bits.  Split products take (32, 2).
  for (int g = 0; g < NU; ++g) {
    const int64_t tot = total_of(jobsA[g]);
    if (tot == 0) continue;
    int cfg = ex.split ? 3 : 0;
    if (!ex.split && ctx->autotune) {
      static const int64_t slots = [] {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return 2 * (int64_t)std::max(cus, 1);
      }();
      const int64_t ntp = std::min(tot, 2 * slots);
      auto lg = [](int64_t v) { int b = 0; while (v > 1) { v >>= 1; ++b; } return b; };
      const std::string key = "krg_f32_persistent u" + std::to_string(u_of[g]) + " tiles2^" + std::to_string(lg(tot));
      static const char* const cfgs[3] = {"chunk16x2", "chunk16x3", "chunk32x2"};
      cfg = autotune_pick(ex, key, 3, cfgs, [&](int i) {
        krg_persistent_launch(ex, bp.jobs + offA[g], (int)jobsA[g].size(), ntp, bp.counter, 0.0, 0.0, u_of[g], i);
      });
    }
    krg_persistent_launch(ex, bp.jobs + offA[g], (int)jobsA[g].size(), tot, bp.counter, flopsA[g], 0.0, u_of[g], cfg);
  }
  for (const auto& a : missA) krg<float, float>(ex, a);
  // they accumulate onto phase A's blocks only, so their place among phase B does not matter
  for (const auto& a : pdiag) krg_pairdiag_gemm(ex, a, bp.pdws);
  for (int g = 0; g < NU; ++g)
    krg_persistent_launch(ex, bp.jobs + offB[g], (int)jobsB[g].size(), total_of(jobsB[g]), bp.counter, flopsB[g],
                          0.0, u_of[g], ex.split ? 3 : 0);
  for (const auto& a : missB) krg<float, float>(ex, a);
  return finish(ex, "hess_batched");
}
