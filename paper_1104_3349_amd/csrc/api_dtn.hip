// C-ABI of the learned interface correction (an extension beyond the paper)
// and of the judged solve that accepts it only when the FP64 GMRES true
// residual reaches the tolerance.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <random>

#include "precond.h"

using namespace addns;


namespace {

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

constexpr char kTag[8] = {'A', 'D', 'D', 'N', 'S', 'D', 'T', 'N'};

// Full-data gradient (scale 1/count) and loss sum, FP32, fixed order.
double full_grad(const float* d_img, const float* X, const float* Y, const float* M, int64_t count, float* d_grad,
                 DevBuf& gpart, DevBuf& lpart, hipStream_t s) {
  const int NP = mlp_param_count();
  const int nwg = mlp_grad_groups(count);
  if (gpart.bytes < sizeof(float) * (size_t)nwg * NP) gpart.alloc(sizeof(float) * (size_t)nwg * NP);
  if (lpart.bytes < sizeof(float) * (size_t)nwg) lpart.alloc(sizeof(float) * nwg);
  launch_mlp_grad(d_img, X, Y, M, nullptr, count, 1.0f / (float)count, gpart.as<float>(), lpart.as<float>(), s);
  launch_mlp_reduce_adam(gpart.as<float>(), nwg, d_grad, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, 0, 0, 1, 1, s);
  std::vector<float> l(nwg);
  ADDNS_HIP(hipMemcpyAsync(l.data(), lpart.p, sizeof(float) * nwg, hipMemcpyDeviceToHost, s));
  ADDNS_HIP(hipStreamSynchronize(s));
  double sum = 0.0;
  for (float v : l) sum += v;
  return sum;
}

}  // namespace

extern "C" {

int addns_dtn_param_count(void) { return mlp_param_count(); }

int addns_dtn_samples(addns_precond_t pc, float* d_X, float* d_Y, float* d_M, int64_t cap, int64_t* count,
                      void* stream) {
  return guarded("addns_dtn_samples", [&]() -> int {
    if (!pc || !count) throw ArgError("null argument");
    const int64_t n = (int64_t)pc->plan.smp_row.size();
    *count = n;
    if (!d_X && !d_Y && !d_M) return ADDNS_OK;  // size query
    require_factors(pc);
    if (pc->schur_mode == ADDNS_SCHUR_LEARNED) throw ArgError("a LEARNED preconditioner has no teacher blocks");
    if ((d_Y == nullptr) != (d_M == nullptr)) throw ArgError("Y and M go together");
    if (d_Y && pc->plan.overlap > 0) throw ArgError("targets need non-overlapped teacher blocks");
    if (cap < n) throw ArgError("capacity smaller than the sample count");
    hipStream_t s = as_stream(stream);
    if (n > 0 && !pc->smp_row.p) {  // sample table uploaded on first use
      pc->smp_row.upload(pc->plan.smp_row, s);
      pc->smp_nb.upload(pc->plan.smp_nb, s);
      pc->smp_loc.upload(pc->plan.smp_loc, s);
    }
    if (d_X)
      launch_dtn_features(n, pc->smp_row.as<int32_t>(), pc->smp_nb.as<int32_t>(), pc->cp_rowptr.as<int32_t>(),
                          pc->cp_colidx.as<int32_t>(), pc->cp_vals.as<double>(), pc->perm.as<int32_t>(),
                          pc->R.as<double>(), d_X, s);
    if (d_Y)
      launch_dtn_targets(n, pc->smp_loc.as<int64_t>(), pc->schur_S.as<double>(), pc->g_copy.as<double>(), d_Y, d_M, s);
    ADDNS_HIP(hipGetLastError());
    return ADDNS_OK;
  });
}

int addns_dtn_forward(const float* h_weights, const float* d_X, float* d_P, int64_t count, int32_t bf16,
                      void* stream) {
  return guarded("addns_dtn_forward", [&]() -> int {
    if (!h_weights || !d_X || !d_P || count < 0) throw ArgError("null argument");
    hipStream_t s = as_stream(stream);
    DevBuf w, img;
    w.alloc(sizeof(float) * mlp_param_count());
    img.alloc(sizeof(float) * mlp_image_floats());
    ADDNS_HIP(hipMemcpyAsync(w.p, h_weights, sizeof(float) * mlp_param_count(), hipMemcpyHostToDevice, s));
    launch_mlp_image(w.as<float>(), img.as<float>(), s);
    launch_mlp_forward(img.as<float>(), d_X, d_P, count, bf16, s);
    ADDNS_HIP(hipStreamSynchronize(s));
    return ADDNS_OK;
  });
}

int addns_dtn_grad(const float* h_weights, const float* d_X, const float* d_Y, const float* d_M, int64_t count,
                   float* h_grad, double* loss, void* stream) {
  return guarded("addns_dtn_grad", [&]() -> int {
    if (!h_weights || !d_X || !d_Y || !d_M || !h_grad || count < 1) throw ArgError("null argument");
    hipStream_t s = as_stream(stream);
    const int NP = mlp_param_count();
    DevBuf w, img, g, gp, lp;
    w.alloc(sizeof(float) * NP);
    img.alloc(sizeof(float) * mlp_image_floats());
    g.alloc(sizeof(float) * NP);
    ADDNS_HIP(hipMemcpyAsync(w.p, h_weights, sizeof(float) * NP, hipMemcpyHostToDevice, s));
    launch_mlp_image(w.as<float>(), img.as<float>(), s);
    const double l = full_grad(img.as<float>(), d_X, d_Y, d_M, count, g.as<float>(), gp, lp, s);
    ADDNS_HIP(hipMemcpyAsync(h_grad, g.p, sizeof(float) * NP, hipMemcpyDeviceToHost, s));
    ADDNS_HIP(hipStreamSynchronize(s));
    if (loss) *loss = l / (double)count;
    return ADDNS_OK;
  });
}

int addns_dtn_train(const float* d_X, const float* d_Y, const float* d_M, int64_t count,
                    const addns_dtn_params* hp, float* h_weights, double* h_loss, void* stream) {
  return guarded("addns_dtn_train", [&]() -> int {
    if (!d_X || !d_Y || !d_M || !hp || !h_weights || count < 1) throw ArgError("null argument");
    if (hp->epochs < 0 || hp->batch < 1 || !(hp->lr > 0.0f)) throw ArgError("epochs >= 0, batch >= 1, lr > 0");
    hipStream_t s = as_stream(stream);
    const int NP = mlp_param_count();
    std::mt19937_64 rng((uint64_t)hp->seed);
    std::vector<float> w0(NP, 0.0f);
    if (hp->init_given) {
      std::copy(h_weights, h_weights + NP, w0.begin());
    } else {  // uniform He initialisation, zero biases
      auto fill = [&](int off, int rows, int cols, float gain) {
        std::uniform_real_distribution<float> u(-1.0f, 1.0f);
        const float a = gain * std::sqrt(3.0f / (float)cols);
        for (int i = 0; i < rows * cols; ++i) w0[off + i] = a * u(rng);
      };
      fill(0, 64, 7, std::sqrt(2.0f));
      fill(64 * 7 + 64, 64, 64, std::sqrt(2.0f));
      fill(64 * 7 + 64 + 64 * 64 + 64, 5, 64, 1.0f);
    }
    DevBuf w, img, m1, m2, grad, gp, lp, idx;
    w.alloc(sizeof(float) * NP);
    img.alloc(sizeof(float) * mlp_image_floats());
    m1.alloc(sizeof(float) * NP);
    m2.alloc(sizeof(float) * NP);
    grad.alloc(sizeof(float) * NP);
    ADDNS_HIP(hipMemcpyAsync(w.p, w0.data(), sizeof(float) * NP, hipMemcpyHostToDevice, s));
    launch_mlp_image(w.as<float>(), img.as<float>(), s);
    ADDNS_HIP(hipMemsetAsync(m1.p, 0, sizeof(float) * NP, s));
    ADDNS_HIP(hipMemsetAsync(m2.p, 0, sizeof(float) * NP, s));
    const int64_t B = hp->batch;
    const int nwg_max = mlp_grad_groups(B);
    gp.alloc(sizeof(float) * (size_t)nwg_max * NP);
    lp.alloc(sizeof(float) * nwg_max);
    std::vector<int32_t> perm(count);
    idx.alloc(sizeof(int32_t) * count);
    const float b1 = hp->beta1, b2 = hp->beta2, eps = hp->eps;
    int64_t step = 0;
    for (int ep = 0; ep < hp->epochs; ++ep) {
      std::iota(perm.begin(), perm.end(), 0);
      std::shuffle(perm.begin(), perm.end(), rng);
      ADDNS_HIP(hipMemcpyAsync(idx.p, perm.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
      ADDNS_HIP(hipStreamSynchronize(s));  // perm is reused next epoch
      for (int64_t off = 0; off < count; off += B) {
        const int64_t nb = std::min(B, count - off);
        const int nwg = mlp_grad_groups(nb);
        ++step;
        launch_mlp_grad(img.as<float>(), d_X, d_Y, d_M, idx.as<int32_t>() + off, nb, 1.0f / (float)nb, gp.as<float>(),
                        lp.as<float>(), s);
        launch_mlp_reduce_adam(gp.as<float>(), nwg, grad.as<float>(), w.as<float>(), img.as<float>(), m1.as<float>(),
                               m2.as<float>(), 1,
                               hp->lr, b1, b2, eps, 1.0f - std::pow(b1, (float)step),
                               1.0f - std::pow(b2, (float)step), s);
      }
      if (h_loss) {
        DevBuf g2, gp2, lp2;
        g2.alloc(sizeof(float) * NP);
        h_loss[ep] = full_grad(img.as<float>(), d_X, d_Y, d_M, count, g2.as<float>(), gp2, lp2, s) / (double)count;
      }
    }
    ADDNS_HIP(hipMemcpyAsync(h_weights, w.p, sizeof(float) * NP, hipMemcpyDeviceToHost, s));
    ADDNS_HIP(hipStreamSynchronize(s));
    return ADDNS_OK;
  });
}

int addns_dtn_save(const char* path, const float* h_weights) {
  return guarded("addns_dtn_save", [&]() -> int {
    if (!path || !h_weights) throw ArgError("null argument");
    std::FILE* f = std::fopen(path, "wb");
    if (!f) throw ArgError(std::string("cannot open ") + path + " for writing");
    const int32_t np = mlp_param_count();
    bool ok = std::fwrite(kTag, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 &&
              std::fwrite(h_weights, 4, (size_t)np, f) == (size_t)np;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw ArgError(std::string("short write to ") + path);
    return ADDNS_OK;
  });
}

int addns_dtn_load(const char* path, float* h_weights) {
  return guarded("addns_dtn_load", [&]() -> int {
    if (!path || !h_weights) throw ArgError("null argument");
    std::FILE* f = std::fopen(path, "rb");
    if (!f) throw ArgError(std::string("cannot open ") + path);
    char tag[8];
    int32_t np = 0;
    const int32_t want = mlp_param_count();
    bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kTag, 8) == 0 && std::fread(&np, 4, 1, f) == 1 &&
              np == want;
    std::vector<float> w(ok ? want : 0);
    ok = ok && std::fread(w.data(), 4, (size_t)want, f) == (size_t)want;
    std::fclose(f);
    if (!ok) throw ArgError(std::string(path) + " is not a weights file of this network");
    std::copy(w.begin(), w.end(), h_weights);
    return ADDNS_OK;
  });
}

int addns_gmres_solve_judged(addns_precond_t learned, addns_precond_t plain, const double* d_b, double* d_x,
                             const addns_gmres_opts* opts, addns_gmres_result* res, int32_t* accepted, void* stream) {
  return guarded("addns_gmres_solve_judged", [&]() -> int {
    if (!learned || !plain || !d_b || !d_x || !opts || !res || !accepted) throw ArgError("null argument");
    require_factors(learned);
    require_factors(plain);
    if (learned->plan.N != plain->plan.N) throw ArgError("the two preconditioners differ in size");
    hipStream_t s = as_stream(stream);
    const int32_t N = plain->plan.N;
    DevBuf x0;
    if (opts->use_x0) {
      x0.alloc(sizeof(double) * N);
      ADDNS_HIP(hipMemcpyAsync(x0.p, d_x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    }
    int code = addns_gmres_solve(learned, d_b, d_x, opts, res, stream);
    if (code == ADDNS_OK && res->converged) {
      *accepted = 1;
      return ADDNS_OK;
    }
    if (code != ADDNS_OK && code != ADDNS_ERR_NOCONV) return code;
    *accepted = 0;  // the learned form missed the tolerance: solve with the plain method
    if (opts->use_x0) ADDNS_HIP(hipMemcpyAsync(d_x, x0.p, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    return addns_gmres_solve(plain, d_b, d_x, opts, res, stream);
  });
}

}  // extern "C"
