// Batched products.  A batch is planned on the host, grouped into size
// classes by transform length, given one workspace per product, and its
// descriptors are copied to the device once; then each class runs as one
// launch of the whole-product kernel (short lengths), or as five launches
// (forward columns, the fused rows, inverse columns, the two recovery
// passes) covering all of its products.  A batch of P products in c
// classes needs at most 5c launches instead of up to 5P.
#include <dmul.h>

#include <algorithm>
#include <map>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

namespace dmi {

void BatchEngine::drop_graphs() {
  for (auto& kv : graphs_) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.descs) (void)hipFree(kv.second.descs);
  }
  graphs_.clear();
}

BatchEngine::~BatchEngine() {
  drop_graphs();
  for (int i = 0; i < kSideStreams; ++i) {
    if (side_[i]) (void)hipStreamDestroy(side_[i]);
    if (join_[i]) (void)hipEventDestroy(join_[i]);
  }
  if (fork_) (void)hipEventDestroy(fork_);
  if (ws_) (void)hipFree(ws_);
  if (sync_) (void)hipFree(sync_);
  if (d_desc_) (void)hipFree(d_desc_);
  if (h_desc_) (void)hipHostFree(h_desc_);
  if (copied_) (void)hipEventDestroy(copied_);
}

int BatchEngine::ensure_side_streams() {
  if (fork_) return DMUL_OK;
  hipError_t e = hipSuccess;
  for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&side_[i], hipStreamNonBlocking);   // default priority
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join_[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork_, hipEventDisableTiming);
  if (e != hipSuccess) {
    for (int i = 0; i < kSideStreams; ++i) {
      if (side_[i]) (void)hipStreamDestroy(side_[i]);
      if (join_[i]) (void)hipEventDestroy(join_[i]);
      side_[i] = nullptr;
      join_[i] = nullptr;
    }
    if (fork_) (void)hipEventDestroy(fork_);
    fork_ = nullptr;
    return from_hip(e);
  }
  return DMUL_OK;
}

int BatchEngine::reserve(dmul_ctx* ctx, size_t ws_words, size_t sync_words, size_t ndesc) {
  const bool grow = ws_words > ws_words_ || sync_words > sync_words_ || ndesc > desc_cap_;
  if (!grow) return DMUL_OK;
  if (ctx->budget && ws_words * sizeof(uint64_t) > ctx->budget) return DMUL_ENOMEM;
  // every growth frees buffers (a wait for the whole device): the small
  // arrays grow by doubling; the workspaces exactly, since they are large
  // and bounded by the budget
  if (sync_words > sync_words_) sync_words = std::max(sync_words, 2 * sync_words_);
  if (ndesc > desc_cap_) ndesc = std::max<size_t>(std::max<size_t>(ndesc, 2 * desc_cap_), 1024);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return from_hip(e);
  drop_graphs();   // captured batches point into the buffers being replaced
  if (ws_words > ws_words_) {
    if (ws_) (void)hipFree(ws_);
    ws_ = nullptr;
    ws_words_ = 0;
    e = hipMalloc(&ws_, ws_words * sizeof(uint64_t));
    if (e != hipSuccess) return from_hip(e);
    ws_words_ = ws_words;
  }
  if (sync_words > sync_words_) {
    if (sync_) (void)hipFree(sync_);
    sync_ = nullptr;
    sync_words_ = 0;
    e = hipMalloc(&sync_, sync_words * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(sync_, 0, sync_words * sizeof(uint32_t));
    if (e != hipSuccess) return from_hip(e);
    sync_words_ = sync_words;
  }
  if (ndesc > desc_cap_) {
    if (d_desc_) (void)hipFree(d_desc_);
    if (h_desc_) (void)hipHostFree(h_desc_);
    d_desc_ = nullptr;
    h_desc_ = nullptr;
    desc_cap_ = 0;
    e = hipMalloc(&d_desc_, ndesc * sizeof(ProdDesc));
    if (e == hipSuccess) e = hipHostMalloc(&h_desc_, ndesc * sizeof(ProdDesc), hipHostMallocDefault);
    if (e != hipSuccess) return from_hip(e);
    desc_cap_ = ndesc;
  }
  return DMUL_OK;
}

int BatchEngine::run(dmul_ctx* ctx, size_t count, const uint64_t* const* a, const size_t* na,
                     const dmul_spectrum* const* sa, const uint64_t* const* b, const size_t* nb,
                     const dmul_spectrum* const* sb, uint64_t* const* out, int32_t* status,
                     unsigned flags, int* status_dev) {
  if (!copied_) {
    if (hipEventCreateWithFlags(&copied_, hipEventDisableTiming) != hipSuccess) return DMUL_EDEVICE;
  }
  auto spec_a = [&](size_t i) { return sa ? sa[i] : nullptr; };
  auto spec_b = [&](size_t i) { return sb ? sb[i] : nullptr; };
  // hipGraph replay: a batch identical to a captured one (same operands,
  // outputs, sizes, spectra, flags, status words) relaunches the captured
  // kernel sequence without planning again.  Captured graphs are dropped
  // whenever the engine's buffers or the tuning change.  The legacy null
  // stream cannot be captured, so graphs need a created stream.
  bool graph = (flags & DMUL_FLAG_GRAPH) && ctx->stream != nullptr && !ctx->prof && !ctx->timing;
  uint64_t sig = 1469598103934665603ULL;
  std::vector<uint64_t> key;
  if (graph) {
    key.reserve(3 + 13 * count);
    key.push_back(count);
    key.push_back(flags);
    key.push_back((uint64_t)status_dev);
    auto spec = [&key](const dmul_spectrum* s) {
      key.push_back(s ? (uint64_t)s->dev : 0);
      key.push_back(s ? s->na : 0);
      key.push_back(s ? s->pl.N : 0);
      key.push_back(s ? (uint64_t)s->pl.k : 0);
    };
    for (size_t i = 0; i < count; ++i) {
      key.push_back((uint64_t)a[i]);
      key.push_back(na[i]);
      key.push_back((uint64_t)b[i]);
      key.push_back(nb[i]);
      key.push_back((uint64_t)out[i]);
      spec(spec_a(i));
      spec(spec_b(i));
    }
    for (uint64_t v : key) sig = (sig ^ v) * 1099511628211ULL;
    auto it = graphs_.find(sig);
    if (it != graphs_.end() && it->second.key == key) {
      for (size_t i = 0; i < count; ++i) {     // empty operands never enter a graph
        if (na[i] == 0 || nb[i] == 0) {
          const hipError_t e = launch_zero(out[i], na[i] + nb[i], ctx->stream);
          if (e != hipSuccess) return from_hip(e);
        }
      }
      if (hipEventRecord(copied_, ctx->stream) != hipSuccess) return DMUL_EDEVICE;
      return from_hip(hipGraphLaunch(it->second.exec, ctx->stream));
    }
  }
  // completion timing: every product starts at the batch's start event and
  // gets its size class's completion event below
  size_t tbase = 0;
  if (ctx->timing) {
    ctx->timing->start(ctx->stream);
    tbase = ctx->timing->done.size();
    ctx->timing->done.resize(tbase + count, 0);
  }
  // plan, and group the products by transform length (and whether cached
  // spectra stand in for operands: those never take the one-workgroup kernel)
  std::vector<PlanDev> plans(count);
  std::map<std::pair<uint64_t, int>, std::vector<uint32_t>> classes;
  size_t ws_words = 0, sync_words = 0, nvalid = 0;
  for (size_t i = 0; i < count; ++i) {
    if (na[i] == 0 || nb[i] == 0) {
      const hipError_t e = launch_zero(out[i], na[i] + nb[i], ctx->stream);
      if (e != hipSuccess) return from_hip(e);
      continue;
    }
    const int rc = spectrum_plan(ctx->device, spec_a(i), na[i], spec_b(i), nb[i],
                                 flags & (DMUL_FLAG_K_MASK | DMUL_FLAG_POW2), &plans[i]);
    if (rc) {
      status[i] = rc;
      graph = false;     // a replay would not report this product's error
      continue;
    }
    classes[{plans[i].N, (spec_a(i) || spec_b(i)) ? 1 : 0}].push_back((uint32_t)i);
    ws_words += workspace_words(plans[i]);
    sync_words += recover_blocks(plans[i], false) + 1;
    ++nvalid;
  }
  if (nvalid == 0) return DMUL_OK;
  sync_words += kQueueTiers;          // the queue heads of the persistent launches
  int rc = reserve(ctx, ws_words, sync_words, nvalid);
  if (rc) {
    for (auto& kv : classes)
      for (uint32_t i : kv.second) status[i] = rc;
    return rc == DMUL_EDEVICE ? rc : DMUL_OK;
  }
  // the staging buffer may still feed the previous batch's copy
  if (hipEventSynchronize(copied_) != hipSuccess) return DMUL_EDEVICE;
  size_t wofs = 0, sofs = 0, di = 0;
  // tier >= 0: the class takes the whole-product kernel through the
  // persistent launch of its tier
  struct Cls { PlanDev p0; int spectra; size_t first, n; Shape sh; const std::vector<uint32_t>* idx; int tier; };
  std::vector<Cls> cls;
  for (auto& kv : classes) {
    const PlanDev& p0 = plans[kv.second[0]];
    Cls c{p0, kv.first.second, 0, kv.second.size(), {}, &kv.second, -1};
    if (ctx->tune.queue && !c.spectra && use_small(ctx, p0, c.n)) c.tier = small_tier(p0);
    cls.push_back(c);
  }
  // queued classes first, tier by tier, longest first (the order in which
  // a tier's queue hands out its products); then the others
  std::stable_sort(cls.begin(), cls.end(), [](const Cls& x, const Cls& y) {
    const int tx = x.tier < 0 ? kQueueTiers : x.tier, ty = y.tier < 0 ? kQueueTiers : y.tier;
    if (tx != ty) return tx < ty;
    return x.tier >= 0 && x.p0.N > y.p0.N;
  });
  for (Cls& c : cls) {
    const PlanDev& p0 = c.p0;
    TwiddleSet ctw;                   // tables exist before any capture
    rc = get_twiddles(ctx, p0, &ctw);
    if (rc) return rc;
    c.first = di;
    c.sh.logR = p0.logR;
    c.sh.logC = p0.logC;
    c.sh.rad3 = p0.rad3;
    c.sh.row_iters = row_iters_for(ctx, p0);
    c.sh.any_nonsquare = 0;
    c.sh.max_nblk = 0;
    c.sh.rec_lean = 0;
    for (uint32_t i : *c.idx) {
      ProdDesc& d = h_desc_[di++];
      d.pl = plans[i];
      d.a = a[i];
      d.b = b[i];
      d.out = out[i];
      d.ws = ws_ + wofs;
      d.status = status_dev + i;
      d.rec_sync = sync_ + sofs;
      d.nblk = (uint32_t)recover_blocks(plans[i], false);
      const dmul_spectrum* si = spec_a(i);
      const dmul_spectrum* ti = spec_b(i);
      d.square = (si || ti) ? (si == ti ? 1 : 0) : ((a[i] == b[i] && na[i] == nb[i]) ? 1 : 0);
      d.xs = si ? si->dev : nullptr;
      d.ys = ti ? ti->dev : nullptr;
      d.scale[0] = ctw.scale[0];
      d.scale[1] = ctw.scale[1];
      if (!d.square) c.sh.any_nonsquare = 1;
      c.sh.max_nblk = std::max(c.sh.max_nblk, d.nblk);
      wofs += workspace_words(plans[i]);
      sofs += d.nblk + 1;
    }
  }
  uint32_t* heads = sync_ + sofs;     // one queue head per tier
  ProdDesc* descs = d_desc_;
  if (graph) {
    if (graphs_.size() >= 8) {
      if (hipStreamSynchronize(ctx->stream) != hipSuccess) return DMUL_EDEVICE;
      drop_graphs();
    }
    hipError_t e = hipMalloc(&descs, nvalid * sizeof(ProdDesc));
    if (e != hipSuccess) return from_hip(e);
  }
  hipError_t e = hipMemcpyAsync(descs, h_desc_, nvalid * sizeof(ProdDesc), hipMemcpyHostToDevice,
                                ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(copied_, ctx->stream);
  if (e != hipSuccess) {
    if (graph) (void)hipFree(descs);
    return from_hip(e);
  }
  // DMUL_POISON: every workspace and map word of the batch starts as
  // garbage (filled here, before any capture begins)
  if (ctx->poison) {
    e = launch_fill32(ws_, 2 * ws_words, kPoison, ctx->stream);
    if (e == hipSuccess) e = launch_fill32(sync_, sync_words, kPoison, ctx->stream);
    if (e != hipSuccess) {
      if (graph) (void)hipFree(descs);
      return from_hip(e);
    }
  }
  // side streams and events exist before any capture begins
  const bool fork = !ctx->prof && cls.size() > 1 && ensure_side_streams() == DMUL_OK;
  if (graph) {
    e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipFree(descs);
      return from_hip(e);
    }
  }
  // the queue heads start at zero for every launch (a fill kernel, so that
  // a captured batch resets them on each replay)
  if (cls.front().tier >= 0) {
    e = launch_fill32(heads, kQueueTiers, 0, ctx->stream);
    if (e != hipSuccess) {
      if (graph) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(ctx->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipFree(descs);
      }
      return from_hip(e);
    }
  }
  Marks* marks = ctx->prof;
  if (ctx->prof) ctx->prof->begin(ctx->stream);
  // classes run concurrently on the side streams (not when profiling, whose
  // per-kernel events assume one stream)
  int nside = 0;
  if (fork) {
    nside = (int)std::min<size_t>(cls.size(), (size_t)side_streams_for(ctx));
    e = hipEventRecord(fork_, ctx->stream);
    for (int i = 0; i < nside && e == hipSuccess; ++i) e = hipStreamWaitEvent(side_[i], fork_, 0);
    if (e != hipSuccess) nside = 0;
  }
  size_t ci = 0;
  // the persistent whole-product launches: one per tier over its classes'
  // products (contiguous descriptors, longest first)
  size_t k = 0;
  while (k < cls.size() && cls[k].tier >= 0 && e == hipSuccess) {
    const int tier = cls[k].tier;
    size_t end = k, count = 0, lds = 0;
    for (; end < cls.size() && cls[end].tier == tier; ++end) {
      count += cls[end].n;
      lds = std::max(lds, small_lds_bytes(cls[end].p0));
    }
    const hipStream_t st = nside ? side_[ci++ % nside] : ctx->stream;
    TwiddleSet tw;                    // its root tables serve every length; the scale is per product
    rc = get_twiddles(ctx, cls[k].p0, &tw);
    if (rc) break;
    Work w{};
    w.many = descs + cls[k].first;
    w.count = (uint32_t)count;
    e = launch_small_queue(w, tier, lds, heads + tier, ctx->cs, tw, ctx->d_div, &ctx->h_div, st, marks);
    if (e == hipSuccess && ctx->timing) {
      const size_t ev = ctx->timing->record(st);
      for (size_t j = k; j < end; ++j)
        for (uint32_t i : *cls[j].idx) ctx->timing->done[tbase + i] = ev;
    }
    k = end;
  }
  for (; k < cls.size() && !rc && e == hipSuccess; ++k) {
    const Cls& c = cls[k];
    const hipStream_t st = nside ? side_[ci++ % nside] : ctx->stream;
    TwiddleSet tw;
    rc = get_twiddles(ctx, c.p0, &tw);
    if (rc) break;
    // grid.z is at most 65535: a very large class goes in several launches
    for (size_t off = 0; off < c.n && e == hipSuccess; off += 65535) {
      Work w{};
      w.many = descs + c.first + off;
      w.count = (uint32_t)std::min<size_t>(65535, c.n - off);
      if (!c.spectra && use_small(ctx, c.p0, c.n)) {
        e = launch_small(w, c.sh, ctx->cs, tw, ctx->d_div, &ctx->h_div, st, marks);
        continue;
      }
      if (c.spectra) {
        e = launch_forward(w, c.sh, ctx->cs, tw, ctx->d_div, st, marks);
        if (e == hipSuccess) e = launch_inverse(w, c.sh, ctx->cs, tw, st, marks);
      } else {
        e = launch_fused(w, c.sh, ctx->cs, tw, ctx->d_div, st, marks);
      }
      if (e == hipSuccess) e = launch_recover(w, c.sh, ctx->cs, ctx->d_div, &ctx->h_div, st, marks);
    }
    if (e != hipSuccess) break;
    if (ctx->timing) {
      const size_t ev = ctx->timing->record(st);
      for (uint32_t i : *c.idx) ctx->timing->done[tbase + i] = ev;
    }
  }
  // join: the context stream continues only after every side stream's classes
  for (int i = 0; i < nside; ++i) {
    const hipError_t ej = hipEventRecord(join_[i], side_[i]);
    const hipError_t ew = ej == hipSuccess ? hipStreamWaitEvent(ctx->stream, join_[i], 0) : ej;
    if (e == hipSuccess) e = ew;
  }
  if (graph) {
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
    if (e == hipSuccess) e = ec;
    Graph entry;
    entry.descs = descs;
    entry.key = std::move(key);
    if (e == hipSuccess && !rc) e = hipGraphInstantiate(&entry.exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e == hipSuccess && !rc) e = hipGraphLaunch(entry.exec, ctx->stream);
    if (e != hipSuccess || rc) {
      if (entry.exec) (void)hipGraphExecDestroy(entry.exec);
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(descs);
      return rc ? rc : from_hip(e);
    }
    auto old = graphs_.find(sig);
    if (old != graphs_.end()) {             // same hash, other batch: the newer one stays
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipGraphExecDestroy(old->second.exec);
      (void)hipFree(old->second.descs);
      graphs_.erase(old);
    }
    graphs_.emplace(sig, std::move(entry));
  }
  if (rc) return rc;
  return from_hip(e);
}

}  // namespace dmi
