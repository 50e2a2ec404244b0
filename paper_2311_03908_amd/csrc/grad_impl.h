// Kinetic-parameter gradient (adjoint) driver of Ctx<T>; included by capi.hip.
//
// Protocol: n_substeps reaction updates of dt_react; every dyn_every updates
// are preceded by one DEM step and a voidage deposit.  The parcel masses stay
// frozen, so the DEM trajectory does not depend on theta: the environment of
// each parcel (gas cell, film resistance) is recorded once per dynamics
// interval, then the reaction recursion runs forward with checkpoints and
// backward with the adjoint.  With grad == NULL the forward runs interval by
// interval and keeps only the current interval's record.
//
// The context's DEM state is snapshotted after a (physically neutral)
// neighbour rebuild, so that the displacements since the rebuild restart
// from zero with it, and restored at the end; the context's reaction state
// is only read.

template <typename T>
int Ctx<T>::grad(const dem_grad_spec *s, const dem_gas *g, const double *theta, double *J, double *gr) {
  if (!s || !J) return fail(DEMRX_EINVAL, "null spec or J");
  if (P.energy_on) return fail(DEMRX_EINVAL, "the gradient protocol is isothermal (energy_on must be 0)");
  if (!gas_ok(g)) return fail(DEMRX_EINVAL, "null gas field");
  if (s->n_substeps < 1 || s->dyn_every < 1 || s->ckpt_every < 1 || !(s->dt_react > 0.0) ||
      !std::isfinite(s->dt_react))
    return fail(DEMRX_EINVAL, "bad gradient spec (n_substeps, dyn_every, ckpt_every >= 1, dt_react > 0)");
  if (theta)
    for (int q = 0; q < 6; q++)
      if (!std::isfinite(theta[q])) return fail(DEMRX_EINVAL, "non-finite theta");
  const bool want = gr != nullptr;
  const int n_sub = s->n_substeps, de = s->dyn_every;
  const int n_int = (n_sub + de - 1) / de;
  const int ck = std::min(s->ckpt_every, n_sub);
  const int n_ck = (n_sub + ck - 1) / ck;
  const int fp32 = s->state_fp32 != 0;
  const size_t ss = fp32 ? sizeof(float) : sizeof(double);
  const size_t N = (size_t)n;
  const int blocks = adjoint_blocks(n);
  const size_t n_rec = want ? (size_t)n_int : 1;

  // ---- scratch layout (one allocation, 256-byte aligned pieces)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t o_cell = take(n_rec * N * 4), o_F = take(n_rec * N * 8);
  const size_t o_ctab = take((size_t)n_gas * 9 * 8), o_dtab = take((size_t)n_gas * P.n_ores * 3 * 8);
  const size_t o_dp = take(N * 8), o_k3 = take(N * 8), o_ore = take(N * 4), o_kind = take(N * 4);
  const size_t o_state = take(4 * N * ss);
  const size_t o_ckpt = want ? take((size_t)n_ck * 4 * N * ss) : 0;
  const size_t o_seg = want ? take((size_t)(ck + 1) * 4 * N * ss) : 0;
  const size_t o_part = take((size_t)blocks * 8 * 8);
  // snapshot of the DEM state
  const size_t o_pos = take(N * sizeof(PosRec)), o_vel = take(N * sizeof(VelRec<T>));
  const size_t o_kcg = take(N * 4), o_tag = take(N * 4), o_sp = take(4 * N * 8);
  const size_t o_wh = take((size_t)3 * kMaxWalls * N * sizeof(T));
  const size_t o_cnt = take(N * 4), o_idx = take((size_t)kMaxNbr * N * 4);
  const size_t o_hist = take((size_t)kMaxNbr * N * sizeof(Spring<T>)), o_mask = take(N * 8);
  const size_t o_eps = take((size_t)n_gas * 8), o_start = take(((size_t)n_keys + 1) * 4);
  const size_t o_xref = take(N * sizeof(float4));
  if (off > gscr.cap) {
    if (gscr.base) (void)hipFree(gscr.base);
    gscr.base = nullptr;
    gscr.cap = 0;
    if (hipMalloc(&gscr.base, off) != hipSuccess) {
      (void)hipGetLastError();
      return fail(DEMRX_ENOMEM, "gradient scratch of " + std::to_string(off) + " bytes failed");
    }
    gscr.cap = off;
  }
  char *B = (char *)gscr.base;

  TRY(rebuild_chain(1, true));  // displacements since the rebuild start from zero
  // ---- snapshot
  struct Cp {
    void *live;
    size_t o, bytes;
  };
  const Dyn<T> &d0 = dyn[cur];
  const Props<T> &p0 = pr;
  const Nbr<T> &b0 = nb;
  const Cp cps[] = {
      {d0.pos, o_pos, N * sizeof(PosRec)}, {d0.vel, o_vel, N * sizeof(VelRec<T>)},
      {p0.kcg, o_kcg, N * 4}, {p0.tag, o_tag, N * 4},
      {p0.nh, o_sp, N * 8}, {p0.nm, o_sp + N * 8, N * 8}, {p0.nw, o_sp + 2 * N * 8, N * 8},
      {p0.nfe, o_sp + 3 * N * 8, N * 8}, {p0.wh, o_wh, (size_t)3 * kMaxWalls * N * sizeof(T)},
      {b0.cnt, o_cnt, N * 4}, {b0.idx, o_idx, (size_t)kMaxNbr * N * 4},
      {b0.hist, o_hist, (size_t)kMaxNbr * N * sizeof(Spring<T>)}, {b0.mask, o_mask, N * 8},
      {eps, o_eps, (size_t)n_gas * 8}, {start, o_start, ((size_t)n_keys + 1) * 4},
      {xref, o_xref, N * sizeof(float4)}};
  for (const Cp &c : cps) HIPCHK(hipMemcpyAsync(B + c.o, c.live, c.bytes, hipMemcpyDeviceToDevice, st));
  const int cur0 = cur;
  const long sc0 = step_count;

  // ---- static tables
  if (theta) HIPCHK(hipMemcpyAsync(theta_d, theta, 6 * sizeof(double), hipMemcpyHostToDevice, st));
  const GasArgs ga = gas_args(g);
  double *ctab = (double *)(B + o_ctab), *dtab = (double *)(B + o_dtab);
  launch_adj_cells(ga, cell_bed, beds, ores, P.n_ores, n_gas, theta ? theta_d : nullptr, ctab, dtab, st);
  AdjArgs a{};
  a.n = n;
  a.n_sub = n_sub;
  a.dyn_every = de;
  a.ckpt_every = ck;
  a.dt = s->dt_react;
  a.rec_cell = (const int32_t *)(B + o_cell);
  a.rec_F = (const double *)(B + o_F);
  a.ctab = ctab;
  a.dtab = dtab;
  a.n_ores = P.n_ores;
  a.dp = (const double *)(B + o_dp);
  a.k3 = (const double *)(B + o_k3);
  a.ore = (const int32_t *)(B + o_ore);
  a.kind = (const int32_t *)(B + o_kind);
  a.state = B + o_state;
  a.ckpt = want ? (void *)(B + o_ckpt) : nullptr;
  a.seg = want ? (void *)(B + o_seg) : nullptr;
  a.part = (double *)(B + o_part);
  if (fp32)
    launch_adj_static<T, float>(dyn[cur], pr, ores, n, (double *)(B + o_dp), (double *)(B + o_k3),
                                (int32_t *)(B + o_ore), (int32_t *)(B + o_kind), (float *)a.state, st);
  else
    launch_adj_static<T, double>(dyn[cur], pr, ores, n, (double *)(B + o_dp), (double *)(B + o_k3),
                                 (int32_t *)(B + o_ore), (int32_t *)(B + o_kind), (double *)a.state, st);
  HIPCHK(hipGetLastError());

  // ---- dynamics intervals: one DEM step, the voidage deposit, the record
  int r = DEMRX_OK;
  for (int k = 0; k < n_int && r == DEMRX_OK; k++) {
    r = gas_table(g);
    if (r == DEMRX_OK) r = step_checked();
    if (r == DEMRX_OK) r = couple(g, nullptr);
    if (r != DEMRX_OK) break;
    const size_t slot = want ? (size_t)k : 0;
    launch_adj_record<T>(dyn[cur], pr, ga, eps, beds, n, (int32_t *)(B + o_cell) + slot * N,
                         (double *)(B + o_F) + slot * N, st);
    if (!want) {  // plain forward: this interval's substeps now
      AdjArgs f = a;
      f.k_base = k;
      f.s_begin = k * de;
      f.s_end = std::min(n_sub, (k + 1) * de);
      f.part = k == n_int - 1 ? a.part : nullptr;
      launch_adjoint_forward(f, fp32, st);
    }
    if (hipGetLastError() != hipSuccess) r = fail(DEMRX_EHIP, "adjoint record/forward launch failed");
  }
  std::vector<double> hp((size_t)blocks * 8);
  double num = 0.0, W = 0.0;
  if (r == DEMRX_OK && want) {
    AdjArgs f = a;
    f.k_base = 0;
    f.s_begin = 0;
    f.s_end = n_sub;
    launch_adjoint_forward(f, fp32, st);
    if (hipGetLastError() != hipSuccess) r = fail(DEMRX_EHIP, "adjoint forward launch failed");
  }
  if (r == DEMRX_OK) {
    if (hipMemcpyAsync(hp.data(), a.part, hp.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      r = fail(DEMRX_EHIP, "adjoint partial sums");
    for (int b = 0; b < blocks; b++) {
      num += hp[(size_t)b * 8];
      W += hp[(size_t)b * 8 + 1];
    }
    if (r == DEMRX_OK && !(W > 0.0)) r = fail(DEMRX_EINVAL, "zero total iron (no parcels carry iron)");
  }
  if (r == DEMRX_OK && want) {
    AdjArgs bw = a;
    bw.k_base = 0;
    bw.inv_W = 1.0 / W;
    launch_adjoint_backward(bw, fp32, st);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hp.data(), a.part, hp.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      r = fail(DEMRX_EHIP, "adjoint backward");
    for (int q = 0; q < 6; q++) {
      double t = 0.0;
      for (int b = 0; b < blocks; b++) t += hp[(size_t)b * 8 + 2 + q];
      gr[q] = t;
    }
  }
  if (r == DEMRX_OK) *J = num / W;

  // ---- restore the DEM state
  cur = cur0;
  step_count = sc0;
  built = true;
  dep_fresh = false;
  chain_step = -1;
  const Dyn<T> &d1 = dyn[cur];
  const Props<T> &p1 = pr;
  const Nbr<T> &b1 = nb;
  void *lives[] = {d1.pos, d1.vel, p1.kcg, p1.tag, p1.nh, p1.nm, p1.nw, p1.nfe, p1.wh,
                   b1.cnt, b1.idx, b1.hist, b1.mask, eps, start, xref};
  for (size_t q = 0; q < sizeof(cps) / sizeof(cps[0]); q++)
    HIPCHK(hipMemcpyAsync(lives[q], B + cps[q].o, cps[q].bytes, hipMemcpyDeviceToDevice, st));
  launch_fill_u32(dslot, 0u, 2 * kSlots * kSlotPad, st);
  HIPCHK(hipGetLastError());
  const int rs = sync();
  return r != DEMRX_OK ? r : rs;
}
