// Batches of independent instances (meshes of different sizes, polynomial
// orders and flow parameters): one context per polynomial order holds the
// disjoint union of its instances' elements, with per-element instance
// indices and per-instance gas parameters, eps, dt a^mm and active flags, so
// that every kernel launch serves all instances of that order.  GMRES,
// Newton and SDIRK run in lockstep over the instances with per-instance
// scalars and masks; each instance goes through exactly the operations of a
// single-instance run (segmented reductions use the same partition), so its
// result equals its solo run.
// Included into dgj_lib.hip (uses its helpers).

namespace {

__global__ void k_dot_seg(const double* __restrict__ x, const double* __restrict__ y, const long* __restrict__ off,
                          const int* __restrict__ active, double* __restrict__ part) {
  __shared__ double red[16];
  const int inst = blockIdx.y;
  if (active && !active[inst]) return;
  const long o = off[inst], n = off[inst + 1] - o;
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s += x[o + i] * y[o + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(long)inst * gridDim.x + blockIdx.x] = s;
}

__global__ void k_reduce_seg(const double* __restrict__ part, int np, const int* __restrict__ active,
                             double* __restrict__ out, int slot, int op) {
  __shared__ double red[16];
  const int inst = blockIdx.x;
  if (active && !active[inst]) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[(long)inst * np + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[inst * 64 + slot] = op == 1 ? sqrt(s) : s;
}

// y += sgn * hs[inst][slot] * x  (masked)
__global__ void k_axpy_seg(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ hs, int slot,
                           double sgn, const int* __restrict__ inst, int nb, const int* __restrict__ active, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ii = inst[i / nb];
    if (active && !active[ii]) continue;
    const double a = sgn * hs[ii * 64 + slot];
    y[i] += a * x[i];
  }
}
// y = a x + b y with a = hs[inst][slot] (hs null: a = a0), masked; kmax: skip instances with kused <= slot
__global__ void k_axpby_seg(double* __restrict__ y, double a0, const double* __restrict__ hs, int slot,
                            const double* __restrict__ x, double b, const int* __restrict__ inst, int nb,
                            const int* __restrict__ active, const int* __restrict__ kused, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ii = inst[i / nb];
    if (active && !active[ii]) continue;
    if (kused && slot >= kused[ii]) continue;
    const double a = hs ? hs[ii * 64 + slot] : a0;
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
  }
}
// y = x / hs[inst][slot] (masked)
__global__ void k_div_seg(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ hs, int slot,
                          const int* __restrict__ inst, int nb, const int* __restrict__ active, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ii = inst[i / nb];
    if (active && !active[ii]) continue;
    y[i] = x[i] / hs[ii * 64 + slot];
  }
}
// y = x (+ a z) masked
__global__ void k_copy_seg(double* __restrict__ y, const double* __restrict__ x, double a, const double* __restrict__ z,
                           const int* __restrict__ inst, int nb, const int* __restrict__ active, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ii = inst[i / nb];
    if (active && !active[ii]) continue;
    y[i] = z ? x[i] + a * z[i] : x[i];
  }
}
__global__ void k_zero_seg(double* __restrict__ y, const int* __restrict__ inst, int nb, const int* __restrict__ active,
                           long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ii = inst[i / nb];
    if (active && !active[ii]) continue;
    y[i] = 0.0;
  }
}

// per-instance host state of the lockstep solvers
struct IG {
  // GMRES
  double beta0 = 0, beta = 0;
  int its = 0, kused = 0;
  bool conv = false, stop = false, done = false, in_cycle = false;
  std::vector<double> H, cs, sn, g, y;
  // Newton
  double n0 = 0, nrm = 0, target = 0;
  int nits = 0;
  bool ndone = false, nconv = true, nan = false;
  std::vector<int> gmres_its;
};

struct Batch {
  int n = 0;
  std::vector<dgj_ctx*> g;      // one context per shape
  std::vector<int> grp, loc;    // per instance
  std::vector<long> off;        // per instance offset in the batch vector
  std::vector<long> goff;       // per group offset
  long n_total = 0;
  dgj_solver sv{};
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<std::vector<int>> act;   // per group host copy of the active flags
  std::vector<double> dt_prev;         // per instance dt of the last step
  // hipGraph replay of the Krylov step (own stream: the legacy stream cannot be captured)
  bool use_graphs = true;
  hipStream_t own = nullptr;
  hipStream_t caller = nullptr;
  std::vector<hipGraphExec_t> gexec;               // [k]: Krylov step k of every group, one graph
  std::vector<double*> h_slots;                    // pinned [group][n_inst*64]
  std::vector<int*> h_act;                         // pinned [group][2 n_inst]: normalisation mask, step mask
};

// one Arnoldi step of group c: z = P^-1 V_k, V_{k+1} = J z, MGS against V_0..V_k, ||V_{k+1}||
void arnoldi_body(dgj_ctx* c, int k) {
  if (c->pc_ready) precond_apply(c, c->V[k], c->d_z);
  else hipLaunchKernelGGL(k_copy_seg, dim3(grid_for(c->n)), dim3(256), 0, c->stream, c->d_z, c->V[k], 0.0, nullptr,
                          c->d_inst, c->NB, c->d_active, c->n);
  double* w = c->V[k + 1];
  matvec(c, c->d_ubar, c->d_N, c->d_S, 0.0, c->d_z, 0.0, w);
  for (int i = 0; i <= k; ++i) {
    hipLaunchKernelGGL(k_dot_seg, dim3(RED_BLOCKS, c->n_inst), dim3(RED_THREADS), 0, c->stream, w, c->V[i], c->d_ioff,
                       c->d_active, c->d_part2);
    hipLaunchKernelGGL(k_reduce_seg, dim3(c->n_inst), dim3(RED_THREADS), 0, c->stream, c->d_part2, RED_BLOCKS,
                       c->d_active, c->d_hs, i, 0);
    hipLaunchKernelGGL(k_axpy_seg, dim3(grid_for(c->n)), dim3(256), 0, c->stream, w, c->V[i], c->d_hs, i, -1.0,
                       c->d_inst, c->NB, c->d_active, c->n);
  }
  hipLaunchKernelGGL(k_dot_seg, dim3(RED_BLOCKS, c->n_inst), dim3(RED_THREADS), 0, c->stream, w, w, c->d_ioff,
                     c->d_active, c->d_part2);
  hipLaunchKernelGGL(k_reduce_seg, dim3(c->n_inst), dim3(RED_THREADS), 0, c->stream, c->d_part2, RED_BLOCKS,
                     c->d_active, c->d_hs, k + 1, 1);
}

// Krylov step k of every order group, all on the batch's stream: for k >= 1
// normalise V[k] (mask h_act[gi][0..n): the instances whose step k-1 had no
// breakdown), then with the step mask h_act[gi][n..2n) the Arnoldi step and
// the copy of the new Hessenberg column to the pinned host slots.  The masks
// are read from pinned host memory when the step runs, so one captured graph
// per k serves every replay.
void krylov_step_body(Batch& B, int k) {
  for (size_t gi = 0; gi < B.g.size(); ++gi) {
    dgj_ctx* c = B.g[gi];
    const size_t mb = (size_t)c->n_inst * sizeof(int);
    if (k >= 1) {
      HIPCHK(hipMemcpyAsync(c->d_active, B.h_act[gi], mb, hipMemcpyHostToDevice, c->stream));
      hipLaunchKernelGGL(k_div_seg, dim3(grid_for(c->n)), dim3(256), 0, c->stream, c->V[k], c->V[k], c->d_hs, k,
                         c->d_inst, c->NB, c->d_active, c->n);
    }
    HIPCHK(hipMemcpyAsync(c->d_active, B.h_act[gi] + c->n_inst, mb, hipMemcpyHostToDevice, c->stream));
    arnoldi_body(c, k);
    HIPCHK(hipMemcpyAsync(B.h_slots[gi], c->d_hs, (size_t)c->n_inst * 64 * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
  }
}

// one launch per Krylov step over all order groups: the step's graph
// (captured on first use) or, without graphs, the same launches directly
void krylov_step(Batch& B, int k) {
  if (!B.use_graphs) {
    krylov_step_body(B, k);
    return;
  }
  if ((int)B.gexec.size() <= k) B.gexec.resize(k + 1, nullptr);
  if (!B.gexec[k]) {
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(B.own, hipStreamCaptureModeThreadLocal));
    krylov_step_body(B, k);
    HIPCHK(hipStreamEndCapture(B.own, &graph));
    HIPCHK(hipGraphInstantiate(&B.gexec[k], graph, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(graph));
  }
  HIPCHK(hipGraphLaunch(B.gexec[k], B.own));
}

void drop_graphs(Batch& B) {
  for (auto& x : B.gexec)
    if (x) { (void)hipGraphExecDestroy(x); x = nullptr; }
}

void set_active(dgj_ctx* c, std::vector<int>& h) {
  HIPCHK(hipMemcpyAsync(c->d_active, h.data(), c->n_inst * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// per-instance norms (op 1) or dots (op 0) into d_hs[inst][slot]
void dot_seg(dgj_ctx* c, const double* x, const double* y, int slot, int op) {
  hipLaunchKernelGGL(k_dot_seg, dim3(RED_BLOCKS, c->n_inst), dim3(RED_THREADS), 0, c->stream, x, y, c->d_ioff,
                     c->d_active, c->d_part2);
  hipLaunchKernelGGL(k_reduce_seg, dim3(c->n_inst), dim3(RED_THREADS), 0, c->stream, c->d_part2, RED_BLOCKS,
                     c->d_active, c->d_hs, slot, op);
}
std::vector<double> fetch_slots(dgj_ctx* c, int nslots) {
  std::vector<double> h((size_t)c->n_inst * 64);
  HIPCHK(hipMemcpyAsync(h.data(), c->d_hs, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  (void)nslots;
  return h;
}
void put_slots(dgj_ctx* c, const std::vector<double>& h) {
  HIPCHK(hipMemcpyAsync(c->d_hs, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

#define SEGL(c) dim3(grid_for((c)->n)), dim3(256), 0, (c)->stream

// Lockstep GMRES over the instances of every group; ig[group][local] hold
// per-instance state; on entry the active flags mark the participating
// instances (Newton-active); buffers are the groups' own (u=d_ubar, Nu=d_N,
// S=d_S, b=d_b, x=d_x).
void batch_gmres(Batch& B, std::vector<std::vector<IG>>& ig) {
  const int m = std::max(1, std::min(B.sv.gmres_restart, 60));
  const double rtol = B.sv.gmres_rtol;
  const int maxit = B.sv.gmres_max;
  const int G = (int)B.g.size();
  auto prec = [&](dgj_ctx* c, const double* in, double* out) {
    if (c->pc_ready) precond_apply(c, in, out);
    else hipLaunchKernelGGL(k_copy_seg, SEGL(c), out, in, 0.0, nullptr, c->d_inst, c->NB, c->d_active, c->n);
  };
  std::vector<std::vector<int>> part(G);   // participating instances (entry active set)
  for (int gi = 0; gi < G; ++gi) {
    dgj_ctx* c = B.g[gi];
    part[gi] = B.act[gi];
    for (int i = 0; i < c->n_inst; ++i) {
      IG& s = ig[gi][i];
      s.its = 0; s.conv = false; s.stop = false; s.done = !part[gi][i]; s.kused = 0;
      s.H.assign((m + 1) * m, 0.0); s.cs.assign(m, 0.0); s.sn.assign(m, 0.0); s.g.assign(m + 1, 0.0); s.y.assign(m, 0.0);
    }
    hipLaunchKernelGGL(k_zero_seg, SEGL(c), c->d_x, c->d_inst, c->NB, c->d_active, c->n);
    dot_seg(c, c->d_b, c->d_b, 63, 1);
    auto h = fetch_slots(c, 64);
    for (int i = 0; i < c->n_inst; ++i) {
      if (!part[gi][i]) continue;
      IG& s = ig[gi][i];
      s.beta0 = h[i * 64 + 63];
      if (!std::isfinite(s.beta0)) fail(DGJ_ENAN, "gmres: non-finite right-hand side (instance)");
      if (s.beta0 == 0.0) { s.conv = true; s.done = true; }
    }
  }
  bool first = true;
  while (true) {
    // residual norms and the start of a cycle
    bool any = false;
    for (int gi = 0; gi < G; ++gi) {
      dgj_ctx* c = B.g[gi];
      std::vector<int> a(c->n_inst, 0);
      for (int i = 0; i < c->n_inst; ++i) a[i] = !ig[gi][i].done;
      set_active(c, a);
      const double* rvec = first ? c->d_b : c->d_t2;
      std::vector<double> h;
      if (!first) {
        dot_seg(c, rvec, rvec, 63, 1);
        h = fetch_slots(c, 64);
      }
      std::vector<double> hb((size_t)c->n_inst * 64, 0.0);
      for (int i = 0; i < c->n_inst; ++i) {
        IG& s = ig[gi][i];
        if (s.done) continue;
        s.beta = first ? s.beta0 : h[i * 64 + 63];
        if (!std::isfinite(s.beta)) fail(DGJ_ENAN, "gmres: non-finite residual (instance)");
        if (s.beta <= rtol * s.beta0) { s.conv = true; s.done = true; a[i] = 0; continue; }
        hb[i * 64 + 62] = s.beta;
        std::fill(s.H.begin(), s.H.end(), 0.0);
        std::fill(s.g.begin(), s.g.end(), 0.0);
        s.g[0] = s.beta;
        s.kused = 0;
        s.stop = false;
        s.in_cycle = true;
        any = true;
      }
      set_active(c, a);
      B.act[gi] = a;
      put_slots(c, hb);
      hipLaunchKernelGGL(k_div_seg, SEGL(c), c->V[0], rvec, c->d_hs, 62, c->d_inst, c->NB, c->d_active, c->n);
    }
    first = false;
    if (!any) break;
    // Arnoldi steps in lockstep: one launch (a replayed graph) per step over
    // all order groups, one host sync per step
    for (int k = 0; k < m; ++k) {
      std::vector<int> live(G, 0);
      for (int gi = 0; gi < G; ++gi) {
        dgj_ctx* c = B.g[gi];
        int* a2 = B.h_act[gi] + c->n_inst;   // this step's mask
        for (int i = 0; i < c->n_inst; ++i) {
          a2[i] = B.act[gi][i];
          live[gi] |= B.act[gi][i];
        }
      }
      krylov_step(B, k);
      HIPCHK(hipStreamSynchronize(B.own));
      bool running = false;
      for (int gi = 0; gi < G; ++gi) {
        dgj_ctx* c = B.g[gi];
        int* a = B.h_act[gi];   // next step's normalisation mask
        for (int ii = 0; ii < c->n_inst; ++ii) a[ii] = 0;
        if (!live[gi]) continue;
        const double* h = B.h_slots[gi];
        for (int ii = 0; ii < c->n_inst; ++ii) {
          a[ii] = B.act[gi][ii];
          if (!a[ii]) continue;
          IG& s = ig[gi][ii];
          s.its++;
          auto Hc = [&](int r, int col) -> double& { return s.H[r * m + col]; };
          for (int r = 0; r <= k + 1; ++r) Hc(r, k) = h[ii * 64 + r];
          if (!std::isfinite(Hc(k + 1, k))) fail(DGJ_ENAN, "gmres: non-finite Krylov vector (instance)");
          const bool breakdown = Hc(k + 1, k) == 0.0;
          for (int r = 0; r < k; ++r) {
            double t = s.cs[r] * Hc(r, k) + s.sn[r] * Hc(r + 1, k);
            Hc(r + 1, k) = -s.sn[r] * Hc(r, k) + s.cs[r] * Hc(r + 1, k);
            Hc(r, k) = t;
          }
          double den = std::hypot(Hc(k, k), Hc(k + 1, k));
          s.cs[k] = Hc(k, k) / den;
          s.sn[k] = Hc(k + 1, k) / den;
          Hc(k, k) = den;
          Hc(k + 1, k) = 0.0;
          s.g[k + 1] = -s.sn[k] * s.g[k];
          s.g[k] = s.cs[k] * s.g[k];
          s.kused = k + 1;
          if (breakdown) a[ii] = 0;   // no division below
          if (std::fabs(s.g[k + 1]) <= rtol * s.beta0 || breakdown || s.its >= maxit) {
            s.conv = std::fabs(s.g[k + 1]) <= rtol * s.beta0 || breakdown;
            s.stop = true;
          }
        }
        // the new vector is normalised at the start of the next step (for
        // the instances without breakdown, mask a); stopped instances leave
        for (int ii = 0; ii < c->n_inst; ++ii) {
          if (!B.act[gi][ii]) continue;
          if (ig[gi][ii].stop) B.act[gi][ii] = 0;
          running |= (bool)B.act[gi][ii];
        }
      }
      if (!running) break;
    }
    // solution update of the instances of this cycle: x += P^-1 (V y)
    bool restart_any = false;
    for (int gi = 0; gi < G; ++gi) {
      dgj_ctx* c = B.g[gi];
      std::vector<int> a(c->n_inst, 0);
      std::vector<double> hy((size_t)c->n_inst * 64, 0.0);
      std::vector<int> ku(c->n_inst, 0);
      int kmax = 0;
      for (int ii = 0; ii < c->n_inst; ++ii) {
        IG& s = ig[gi][ii];
        if (!s.in_cycle) continue;
        a[ii] = 1;
        auto Hc = [&](int r, int col) -> double& { return s.H[r * m + col]; };
        for (int r = s.kused - 1; r >= 0; --r) {
          double t = s.g[r];
          for (int j = r + 1; j < s.kused; ++j) t -= Hc(r, j) * s.y[j];
          s.y[r] = t / Hc(r, r);
        }
        for (int r = 0; r < s.kused; ++r) hy[ii * 64 + r] = s.y[r];
        ku[ii] = s.kused;
        kmax = std::max(kmax, s.kused);
      }
      set_active(c, a);
      put_slots(c, hy);
      HIPCHK(hipMemcpyAsync(c->d_kused, ku.data(), c->n_inst * sizeof(int), hipMemcpyHostToDevice, c->stream));
      hipLaunchKernelGGL(k_zero_seg, SEGL(c), c->d_t1, c->d_inst, c->NB, c->d_active, c->n);
      for (int r = 0; r < kmax; ++r)
        hipLaunchKernelGGL(k_axpby_seg, SEGL(c), c->d_t1, 0.0, c->d_hs, r, c->V[r], 1.0, c->d_inst, c->NB,
                           c->d_active, c->d_kused, c->n);
      prec(c, c->d_t1, c->d_z);
      hipLaunchKernelGGL(k_axpby_seg, SEGL(c), c->d_x, 1.0, nullptr, 0, c->d_z, 1.0, c->d_inst, c->NB, c->d_active,
                         nullptr, c->n);
      // instances that finished leave; the others restart with r = b - J x
      std::vector<int> ra(c->n_inst, 0);
      for (int ii = 0; ii < c->n_inst; ++ii) {
        IG& s = ig[gi][ii];
        if (!s.in_cycle) continue;
        s.in_cycle = false;
        if (s.conv || s.stop) s.done = true;
        else { ra[ii] = 1; restart_any = true; }
      }
      set_active(c, ra);
      B.act[gi] = ra;
      matvec(c, c->d_ubar, c->d_N, c->d_S, 0.0, c->d_x, 0.0, c->d_t2);
      hipLaunchKernelGGL(k_copy_seg, SEGL(c), c->d_t2, c->d_b, -1.0, c->d_t2, c->d_inst, c->NB, c->d_active, c->n);
    }
    if (!restart_any) break;
  }
  // restore the participation mask
  for (int gi = 0; gi < G; ++gi) {
    B.act[gi] = part[gi];
    set_active(B.g[gi], B.act[gi]);
  }
}

// Lockstep Newton for the stage with per-instance dt a^mm in d_dtav; u = d_ubar, S = d_S.
void batch_newton(Batch& B, std::vector<std::vector<IG>>& ig) {
  const int G = (int)B.g.size();
  for (int gi = 0; gi < G; ++gi) {
    dgj_ctx* c = B.g[gi];
    B.act[gi].assign(c->n_inst, 1);
    set_active(c, B.act[gi]);
    stage_residual(c, c->d_ubar, c->d_S, 0.0, c->d_N);
    dot_seg(c, c->d_N, c->d_N, 63, 1);
    auto h = fetch_slots(c, 64);
    for (int i = 0; i < c->n_inst; ++i) {
      IG& s = ig[gi][i];
      s.nits = 0; s.ndone = false; s.nconv = true; s.nan = false; s.gmres_its.clear();
      s.n0 = h[i * 64 + 63];
      s.nrm = s.n0;
      s.target = B.sv.newton_rtol * s.n0;
      if (!std::isfinite(s.n0)) { s.nan = true; s.nconv = false; s.ndone = true; }
    }
  }
  while (true) {
    bool any = false;
    for (int gi = 0; gi < G; ++gi) {
      dgj_ctx* c = B.g[gi];
      // ||u|| of the instances still iterating
      std::vector<int> a(c->n_inst, 0);
      for (int i = 0; i < c->n_inst; ++i) a[i] = !ig[gi][i].ndone;
      set_active(c, a);
      dot_seg(c, c->d_ubar, c->d_ubar, 61, 1);
      auto h = fetch_slots(c, 64);
      std::vector<double> eps(c->n_inst, 0.0);
      for (int i = 0; i < c->n_inst; ++i) {
        IG& s = ig[gi][i];
        if (s.ndone) continue;
        const double nu = h[i * 64 + 61];
        if (s.nrm < s.target || s.nrm <= 1e-14 * nu) { s.ndone = true; a[i] = 0; continue; }
        if (s.nits >= B.sv.newton_max) { s.nconv = false; s.ndone = true; a[i] = 0; continue; }
        eps[i] = nu * std::sqrt(EPS_HAT);
        any = true;
      }
      HIPCHK(hipMemcpyAsync(c->d_epsv, eps.data(), c->n_inst * sizeof(double), hipMemcpyHostToDevice, c->stream));
      B.act[gi] = a;
      set_active(c, a);
      hipLaunchKernelGGL(k_axpby_seg, SEGL(c), c->d_b, -1.0, nullptr, 0, c->d_N, 0.0, c->d_inst, c->NB, c->d_active,
                         nullptr, c->n);
    }
    if (!any) break;
    batch_gmres(B, ig);
    for (int gi = 0; gi < G; ++gi) {
      dgj_ctx* c = B.g[gi];
      hipLaunchKernelGGL(k_axpby_seg, SEGL(c), c->d_ubar, 1.0, nullptr, 0, c->d_x, 1.0, c->d_inst, c->NB, c->d_active,
                         nullptr, c->n);
      stage_residual(c, c->d_ubar, c->d_S, 0.0, c->d_N);
      dot_seg(c, c->d_N, c->d_N, 63, 1);
      auto h = fetch_slots(c, 64);
      for (int i = 0; i < c->n_inst; ++i) {
        IG& s = ig[gi][i];
        if (!B.act[gi][i]) continue;
        s.gmres_its.push_back(s.its);
        s.nrm = h[i * 64 + 63];
        s.nits++;
        if (!std::isfinite(s.nrm)) { s.nan = true; s.nconv = false; s.ndone = true; }
      }
    }
  }
}

}  // namespace

struct dgj_batch : Batch {};

extern "C" {

int dgj_batch_create(int32_t n, const dgj_mesh* meshes, const dgj_phys* phys, const dgj_solver* solver,
                     void* hip_stream, dgj_batch** out) {
  if (!out) return DGJ_EINVAL;
  *out = nullptr;
  if (n < 1 || !meshes || !phys || !solver) return DGJ_EINVAL;
  dgj_batch* b = new dgj_batch();
  b->n = n;
  b->sv = *solver;
  b->caller = (hipStream_t)hip_stream;
  int rc = DGJ_OK;
  try {
    HIPCHK(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking));
    b->stream = b->own;
    // groups by (dim, P, nq), in order of first appearance
    std::vector<std::array<int, 3>> keys;
    b->grp.assign(n, -1);
    b->loc.assign(n, -1);
    if (solver->scheme != DGJ_SDIRK2 && solver->scheme != DGJ_SDIRK3)
      throw Status{DGJ_EUNSUPPORTED, "batch: scheme must be SDIRK2 or SDIRK3"};
    if (solver->ortho != 0) throw Status{DGJ_EUNSUPPORTED, "batch: modified Gram-Schmidt only"};
    for (int i = 0; i < n; ++i)
      if (phys[i].viscous != 0) throw Status{DGJ_EUNSUPPORTED, "batch: interior-penalty viscous terms only"};
    for (int i = 0; i < n; ++i) {
      if (meshes[i].geo_nodes || !meshes[i].elem_h || !meshes[i].elem_origin || !meshes[i].face_nbr)
        throw Status{DGJ_EUNSUPPORTED, "batch: instances must be periodic meshes of affine boxes"};
      std::array<int, 3> k = {meshes[i].dim, meshes[i].P, meshes[i].nq};
      auto it = std::find(keys.begin(), keys.end(), k);
      if (it == keys.end()) { keys.push_back(k); b->grp[i] = (int)keys.size() - 1; }
      else b->grp[i] = (int)(it - keys.begin());
    }
    long pos = 0;
    for (size_t gi = 0; gi < keys.size(); ++gi) {
      std::vector<int> members;
      for (int i = 0; i < n; ++i)
        if (b->grp[i] == (int)gi) members.push_back(i);
      const int D = keys[gi][0];
      long E = 0;
      for (int i : members) E += meshes[i].n_elem;
      std::vector<double> org(E * D), h(E * D);
      std::vector<int32_t> nbr(E * 2 * D);
      std::vector<int> inst(E);
      std::vector<long> e0(members.size() + 1, 0);
      long eo = 0;
      for (size_t k = 0; k < members.size(); ++k) {
        const dgj_mesh& ms = meshes[members[k]];
        e0[k] = eo;
        for (long e = 0; e < ms.n_elem; ++e) {
          for (int j = 0; j < D; ++j) {
            org[(eo + e) * D + j] = ms.elem_origin[e * D + j];
            h[(eo + e) * D + j] = ms.elem_h[e * D + j];
          }
          for (int f = 0; f < 2 * D; ++f) {
            const int32_t nb = ms.face_nbr[e * 2 * D + f];
            if (nb < 0 || nb >= ms.n_elem) throw Status{DGJ_EUNSUPPORTED, "batch: boundary faces are not supported"};
            nbr[(eo + e) * 2 * D + f] = (int32_t)(nb + eo);
          }
          inst[eo + e] = (int)k;
        }
        b->loc[members[k]] = (int)k;
        eo += ms.n_elem;
      }
      e0[members.size()] = eo;
      dgj_mesh gm{D, keys[gi][1], keys[gi][2], E, org.data(), h.data(), nbr.data()};
      dgj_ctx* c = nullptr;
      int r = dgj_create(&gm, &phys[members[0]], solver, (void*)b->own, &c);
      if (r != DGJ_OK) throw Status{r, "batch: creating a group context failed"};
      b->g.push_back(c);
      c->n_inst = (int)members.size();
      c->inst_e0 = e0;
      c->h_phs.clear();
      for (int i : members) {
        const dgj_phys& p = phys[i];
        c->h_phs.push_back(Phys{p.gamma, p.Pr, p.Re, p.Ma, p.T_ref_K, p.visc_law, p.flux_mode, p.riemann});
      }
      std::vector<long> ioff(members.size() + 1);
      for (size_t k = 0; k <= members.size(); ++k) ioff[k] = e0[k] * c->NB;
      const int ni = c->n_inst;
      HIPCHK(hipMalloc(&c->d_inst, E * sizeof(int)));
      HIPCHK(hipMalloc(&c->d_phs, ni * sizeof(Phys)));
      HIPCHK(hipMalloc(&c->d_epsv, ni * sizeof(double)));
      HIPCHK(hipMalloc(&c->d_dtav, ni * sizeof(double)));
      HIPCHK(hipMalloc(&c->d_active, ni * sizeof(int)));
      HIPCHK(hipMalloc(&c->d_ioff, (ni + 1) * sizeof(long)));
      HIPCHK(hipMalloc(&c->d_hs, (size_t)ni * 64 * sizeof(double)));
      HIPCHK(hipMalloc(&c->d_part2, (size_t)ni * RED_BLOCKS * sizeof(double)));
      HIPCHK(hipMalloc(&c->d_kused, ni * sizeof(int)));
      std::vector<int> ones(ni, 1);
      std::vector<double> zeros(ni, 0.0);
      HIPCHK(hipMemcpy(c->d_inst, inst.data(), E * sizeof(int), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(c->d_phs, c->h_phs.data(), ni * sizeof(Phys), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(c->d_active, ones.data(), ni * sizeof(int), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(c->d_epsv, zeros.data(), ni * sizeof(double), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(c->d_dtav, zeros.data(), ni * sizeof(double), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(c->d_ioff, ioff.data(), (ni + 1) * sizeof(long), hipMemcpyHostToDevice));
      b->act.push_back(ones);
      double* hs = nullptr;
      int* ha = nullptr;
      HIPCHK(hipHostMalloc(&hs, (size_t)ni * 64 * sizeof(double), hipHostMallocDefault));
      HIPCHK(hipHostMalloc(&ha, (size_t)ni * 2 * sizeof(int), hipHostMallocDefault));
      b->h_slots.push_back(hs);
      b->h_act.push_back(ha);
      b->goff.push_back(pos);
      pos += c->n;
    }
    b->off.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      dgj_ctx* c = b->g[b->grp[i]];
      b->off[i] = b->goff[b->grp[i]] + c->inst_e0[b->loc[i]] * c->NB;
    }
    b->n_total = pos;
    b->off[n] = pos;
    b->dt_prev.assign(n, 0.0);
  } catch (const Status& s) {
    b->err = s.msg;
    rc = s.code;
  } catch (const HipError& h) {
    b->err = hipGetErrorString(h.e);
    rc = DGJ_EHIP;
  }
  if (rc != DGJ_OK) {
    fprintf(stderr, "dgj_batch_create: %s\n", b->err.c_str());
    dgj_batch_destroy(b);
    return rc;
  }
  *out = b;
  return DGJ_OK;
}

int dgj_create_batch(int32_t n, const dgj_mesh* meshes, const dgj_phys* phys, const dgj_solver* solver,
                     void* hip_stream, dgj_batch** out) {
  return dgj_batch_create(n, meshes, phys, solver, hip_stream, out);
}

void dgj_batch_destroy(dgj_batch* b) {
  if (!b) return;
  if (b->own) (void)hipStreamSynchronize(b->own);
  drop_graphs(*b);
  for (auto* c : b->g) dgj_destroy(c);
  for (double* p : b->h_slots)
    if (p) (void)hipHostFree(p);
  for (int* p : b->h_act)
    if (p) (void)hipHostFree(p);
  if (b->own) (void)hipStreamDestroy(b->own);
  delete b;
}

int dgj_batch_set_graphs(dgj_batch* b, int32_t on) {
  if (!b) return DGJ_EINVAL;
  b->use_graphs = on != 0;
  return DGJ_OK;
}

const char* dgj_batch_last_error(const dgj_batch* b) { return b ? b->err.c_str() : "null batch"; }

int dgj_batch_sizes(const dgj_batch* b, int64_t* n_total, int64_t* offsets, int64_t* counts) {
  if (!b) return DGJ_EINVAL;
  if (n_total) *n_total = b->n_total;
  for (int i = 0; i < b->n; ++i) {
    const dgj_ctx* c = b->g[b->grp[i]];
    if (offsets) offsets[i] = b->off[i];
    if (counts) counts[i] = (c->inst_e0[b->loc[i] + 1] - c->inst_e0[b->loc[i]]) * c->NB;
  }
  return DGJ_OK;
}

static int batch_guard(dgj_batch* b, const std::function<int()>& f) {
  try {
    // the batch works on its own stream: wait for the caller's work first and
    // finish before returning
    HIPCHK(hipStreamSynchronize(b->caller));
    int r = f();
    HIPCHK(hipStreamSynchronize(b->own));
    return r;
  } catch (const HipError& h) {
    b->err = std::string("HIP error ") + hipGetErrorString(h.e) + " in " + h.what;
    return DGJ_EHIP;
  } catch (const Status& s) {
    b->err = s.msg;
    return s.code;
  }
}

int dgj_batch_project_tgv(dgj_batch* b, const double* noise, double amp, double* u) {
  if (!b || !u) return DGJ_EINVAL;
  return batch_guard(b, [&]() -> int {
    for (size_t gi = 0; gi < b->g.size(); ++gi) {
      int r = dgj_project_tgv(b->g[gi], noise ? noise + b->goff[gi] : nullptr, amp, u + b->goff[gi]);
      if (r != DGJ_OK) throw Status{r, b->g[gi]->err};
    }
    return DGJ_OK;
  });
}

int dgj_batch_residual(dgj_batch* b, const double* u, double* R) {
  if (!b || !u || !R) return DGJ_EINVAL;
  return batch_guard(b, [&]() -> int {
    for (size_t gi = 0; gi < b->g.size(); ++gi) {
      dgj_ctx* c = b->g[gi];
      std::vector<int> ones(c->n_inst, 1);
      set_active(c, ones);
      residual(c, u + b->goff[gi], R + b->goff[gi]);
    }
    HIPCHK(hipGetLastError());
    return DGJ_OK;
  });
}

int dgj_batch_autotune(dgj_batch* b, const double* u, int32_t reps, int32_t* chosen, int32_t* n_groups) {
  if (!b || !u || reps < 1) return DGJ_EINVAL;
  return batch_guard(b, [&]() -> int {
    for (size_t gi = 0; gi < b->g.size(); ++gi) {
      dgj_ctx* c = b->g[gi];
      std::vector<int> ones(c->n_inst, 1);
      set_active(c, ones);
      autotune(c, u + b->goff[gi], reps, chosen ? chosen + 3 * gi : nullptr, nullptr);
    }
    drop_graphs(*b);   // captured launches hold the old workgroup sizes
    if (n_groups) *n_groups = (int32_t)b->g.size();
    HIPCHK(hipGetLastError());
    return DGJ_OK;
  });
}

int dgj_batch_sdirk_step(dgj_batch* b, double* u, const double* dt, int32_t* newton_its, int32_t* gmres_its) {
  if (!b || !u || !dt) return DGJ_EINVAL;
  for (int i = 0; i < b->n; ++i)
    if (!(dt[i] > 0.0)) return DGJ_EINVAL;
  return batch_guard(b, [&]() -> int {
    double A[DGJ_MAX_STAGES][DGJ_MAX_STAGES], bb[DGJ_MAX_STAGES];
    int s = 0;
    tableau(b->sv.scheme, A, bb, s);
    const int G = (int)b->g.size();
    std::vector<std::vector<IG>> ig(G);
    for (int gi = 0; gi < G; ++gi) ig[gi].resize(b->g[gi]->n_inst);
    // preconditioner: rebuilt for every instance when stale or dt a^mm changed
    for (int gi = 0; gi < G; ++gi) {
      dgj_ctx* c = b->g[gi];
      double* ug = u + b->goff[gi];
      std::vector<int> insts;
      std::vector<double> dta;
      bool stale = !c->pc_ready || c->pc_age >= b->sv.pc_freeze;
      for (int i = 0; i < b->n; ++i)
        if (b->grp[i] == gi && std::fabs(b->dt_prev[i] - dt[i]) > 1e-12 * dt[i]) stale = true;
      if (stale) {
        drop_graphs(*b);   // captured Krylov steps refer to the preconditioner state
        for (int k = 0; k < c->n_inst; ++k) insts.push_back(k);
        for (int i = 0; i < b->n; ++i)
          if (b->grp[i] == gi) dta.push_back(0.0);
        for (int i = 0; i < b->n; ++i)
          if (b->grp[i] == gi) dta[b->loc[i]] = dt[i] * A[0][0];
        precond_build_insts(c, ug, insts, dta);
      }
      copy(c, c->d_un, ug);
    }
    for (int i = 0; i < b->n; ++i) b->dt_prev[i] = dt[i];
    for (int mst = 0; mst < s; ++mst) {
      for (int gi = 0; gi < G; ++gi) {
        dgj_ctx* c = b->g[gi];
        std::vector<double> dta(c->n_inst);
        for (int i = 0; i < b->n; ++i)
          if (b->grp[i] == gi) dta[b->loc[i]] = dt[i] * A[mst][mst];
        HIPCHK(hipMemcpyAsync(c->d_dtav, dta.data(), c->n_inst * sizeof(double), hipMemcpyHostToDevice, c->stream));
        copy(c, c->d_S, c->d_un);
        for (int i = 0; i < mst; ++i) axpby(c, c->d_S, A[mst][i], c->d_E[i], 1.0);
        copy(c, c->d_ubar, c->d_S);
        HIPCHK(hipStreamSynchronize(c->stream));
      }
      batch_newton(*b, ig);
      for (int gi = 0; gi < G; ++gi) {
        dgj_ctx* c = b->g[gi];
        for (int i = 0; i < c->n_inst; ++i) {
          IG& st = ig[gi][i];
          if (st.nan) fail(DGJ_ENAN, "batch stage %d: non-finite residual", mst);
          if (!st.nconv) fail(DGJ_ENOTCONV, "batch stage %d: Newton not converged", mst);
        }
        for (int i = 0; i < b->n; ++i) {
          if (b->grp[i] != gi) continue;
          const IG& st = ig[gi][b->loc[i]];
          if (newton_its) newton_its[i * 4 + mst] = st.nits;
          if (gmres_its) {
            int t = 0;
            for (int x : st.gmres_its) t += x;
            gmres_its[i * 4 + mst] = t;
          }
        }
        std::vector<int> ones(c->n_inst, 1);
        b->act[gi] = ones;
        set_active(c, ones);
        hipLaunchKernelGGL(k_sub_div, dim3(grid_for(c->n)), dim3(256), 0, c->stream, c->d_E[mst], c->d_ubar, c->d_S,
                           A[mst][mst], c->n);
      }
    }
    for (int gi = 0; gi < G; ++gi) {
      dgj_ctx* c = b->g[gi];
      copy(c, c->d_t1, c->d_un);
      for (int i = 0; i < s; ++i) axpby(c, c->d_t1, bb[i], c->d_E[i], 1.0);
      copy(c, u + b->goff[gi], c->d_t1);
      HIPCHK(hipStreamSynchronize(c->stream));
      c->pc_age++;
    }
    return DGJ_OK;
  });
}

}  // extern "C"
