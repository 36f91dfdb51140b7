"""Compound operators (Sec. 4.2) composed from the C-ABI primitives, with all
buffers allocated once so that repeated steps allocate nothing.

WindowAggregation: windowing (partition on the timestamp column) -> per-window
sort of the KPA -> keyed reduction (count, sum, max) -> top-k keys by sum.
SlidingAggregation: the same per key over sliding windows, built from panes
(partitions one slide long, Sec. 4.2 "Windowing").
"""
from __future__ import annotations

import torch

from . import kpa as K


class _Layout:
    def __init__(self, row_bytes, key_off, val_off, val_w, ts_off, ts_w):
        self.row_bytes, self.key_off, self.val_off = row_bytes, key_off, val_off
        self.val_w, self.ts_off, self.ts_w = val_w, ts_off, ts_w


# A staged value column read as 8-byte rows whose only field is the value.
VALUE_COLUMN = _Layout(8, 0, 0, 8, 0, 8)


class WindowAggregation:
    def __init__(self, n, layout, win_len, n_win, algo=K.KPA_SORT_RADIX, k=10, device="cuda",
                 win_origin=0, want=("cnt", "sum", "max"), stage_values=True):
        self.n, self.layout, self.win_len, self.n_win = n, layout, win_len, n_win
        self.algo, self.k, self.origin = algo, k, win_origin
        self.want = tuple(want)
        d = torch.device(device)
        cap = max(n, 1)
        i64 = dict(dtype=torch.int64, device=d)
        i32 = dict(dtype=torch.int32, device=d)
        self.keys = torch.empty(cap, **i64)
        self.rids = torch.empty(cap, **i32)
        self.skeys = torch.empty(cap, **i64)
        self.srids = torch.empty(cap, **i32)
        self.win_off = torch.empty(n_win + 1, **i64)
        self.oob = torch.empty(1, **i64)
        # the value column staged compactly at partition time (8 bytes per row);
        # the reduction gathers from it instead of from the full rows
        self.vals = torch.empty(cap, **i64) if stage_values else None
        self.gkey = torch.empty(cap, **i64)
        self.g = {w: torch.empty(cap, **i64) for w in self.want}
        self.gseg = torch.empty(n_win + 1, **i64)
        self.top_key = torch.empty(n_win * k, **i64)
        self.top_sum = torch.empty(n_win * k, **i64)
        self.top_n = torch.empty(n_win, **i32)
        u8 = dict(dtype=torch.uint8, device=d)
        self.ws_part = torch.empty(
            K._ws_size("kpa_partition_windows_workspace_size", n, n_win), **u8)
        self.ws_sort = torch.empty(max(K.kpa_sort_workspace_size(n, n_win, K.KPA_SORT_RADIX),
                                       K.kpa_sort_workspace_size(n, n_win, algo)), **u8)
        self.ws_red = torch.empty(K._ws_size("kpa_reduce_by_key_workspace_size", n, n_win), **u8)
        self.ws_top = torch.empty(K._ws_size("kpa_topk_by_sum_workspace_size", n, n_win), **u8)
        self.models = K.new_models(n_win, d)
        self.next_models = K.new_models(n_win, d)
        self.stats = K.new_sort_stats(d)
        self.have_models = False

    def step(self, rows, stream=None):
        K.kpa_partition_windows(rows, self.layout, self.win_len, self.n_win,
                                win_origin=self.origin, n=self.n, out_keys=self.keys,
                                out_rids=self.rids, out_win_off=self.win_off, out_oob=self.oob,
                                ws=self.ws_part, stream=stream, out_vals=self.vals)
        algo = self.algo if (self.algo == K.KPA_SORT_RADIX or self.have_models) else K.KPA_SORT_RADIX
        K.kpa_sort_segmented(self.keys, self.rids, self.win_off, n_cap=self.n, algo=algo,
                             models=self.models if algo == K.KPA_SORT_LEARNED else None,
                             stats=self.stats, keys_out=self.skeys, rids_out=self.srids,
                             ws=self.ws_sort, stream=stream)
        if self.algo == K.KPA_SORT_LEARNED:
            # Window w of the next batch is bucketed with the model fitted on
            # window w-1 of this batch (window 0 with this batch's last window):
            # each model comes from an earlier window, never its own data.
            K.kpa_pwl_fit(self.skeys, self.win_off, 1024, models=self.next_models, stream=stream)
            mb = K.PWL_MODEL_BYTES
            # on the step's stream: after the fit, before the next step's sort
            with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
                self.models[mb:].copy_(self.next_models[:-mb])
                self.models[:mb].copy_(self.next_models[-mb:])
            self.have_models = True
        outs = dict(self.g)
        outs["gkey"] = self.gkey
        outs["gseg_off"] = self.gseg
        src, lay = (self.vals, VALUE_COLUMN) if self.vals is not None else (rows, self.layout)
        K.kpa_reduce_by_key(self.skeys, self.srids, self.win_off, src, lay, n_cap=self.n,
                            want=self.want, ws=self.ws_red, stream=stream, outs=outs)
        if "sum" in self.g:
            K.kpa_topk_by_sum(self.gkey, self.g["sum"], self.gseg, k=self.k, g_cap=self.n,
                              ws=self.ws_top, stream=stream,
                              outs={"key": self.top_key, "sum": self.top_sum, "n": self.top_n})


class BatchAggregation:
    """Many substreams' windows at once, one segment each (substream j's rows
    back to back in the arena): extract with the value column staged ->
    batched sort (small / mid / large classes, radix or learned for the large
    ones) -> keyed reduction (count, sum, max) per window.  Every buffer is
    allocated here, so a step can be captured once in a graph and replayed.

    carry_values: True: the sort carries the staged value column beside the
    KPA (8 more bytes read and written per entry and pass) and the reduction
    reads it in KPA order; False: the reduction follows each row id into the
    staged column (a cache-line fetch per entry); None (default): carry on
    the learned route (two scatter passes and the finishing pass) and follow
    the row ids on the radix route (as many passes as key bytes vary).
    Group keys land in the sort's input key array, which is dead once the
    sort ran, and the sums in whichever value array the reduction does not
    read, so results stay valid until the next step (pipe.g after a step).
    """

    def __init__(self, n_rows, n_seg, layout, cfg=None, device="cuda",
                 want=("cnt", "sum", "max"), learned_ws=True, carry_values=None):
        self.n, self.n_seg, self.layout = n_rows, n_seg, layout
        self.cfg = K.kpa_batch_config_default() if cfg is None else cfg
        self.want = tuple(want)
        self.carry = carry_values
        d = torch.device(device)
        cap = max(n_rows, 1)
        i64 = dict(dtype=torch.int64, device=d)
        i32 = dict(dtype=torch.int32, device=d)
        self.keys = torch.empty(cap, **i64)   # no input rids: extract writes none and
        self.vals = torch.empty(cap, **i64)   # the sort takes each entry's position
        self.skeys = torch.empty(cap, **i64)
        self.srids = torch.empty(cap, **i32)
        self.svals = torch.empty(cap, **i64)
        self.seg_off = torch.zeros(n_seg + 1, **i64)
        self.gkey = self.keys
        other = {w: torch.empty(cap, **i64) for w in self.want if w != "sum"}
        # sums: into the value array the reduction does not read
        self._g = {True: dict(other, **({"sum": self.vals} if "sum" in self.want else {})),
                   False: dict(other, **({"sum": self.svals} if "sum" in self.want else {}))}
        self.g = self._g[carry_values is not False]
        self.gseg = torch.empty(n_seg + 1, **i64)
        u8 = dict(dtype=torch.uint8, device=d)
        ws_size = (K.kpa_batch_sort_vals_workspace_size if carry_values is not False
                   else K.kpa_batch_sort_workspace_size)
        sizes = [ws_size(n_rows, n_seg, K.batch_config(large_algo=K.KPA_SORT_RADIX))]
        if learned_ws:
            sizes.append(ws_size(n_rows, n_seg, K.batch_config(large_algo=K.KPA_SORT_LEARNED)))
        self.ws_sort = torch.empty(max(sizes), **u8)
        self.ws_red = torch.empty(K._ws_size("kpa_reduce_by_key_workspace_size", n_rows, n_seg),
                                  **u8)
        self.models = K.new_models(n_seg, d)
        self.next_models = K.new_models(n_seg, d)
        self.stats = K.new_sort_stats(d)

    def set_sizes(self, sizes):
        off = torch.zeros(self.n_seg + 1, dtype=torch.int64)
        off[1:] = torch.cumsum(torch.as_tensor(sizes, dtype=torch.int64), 0)
        if int(off[-1]) > self.n:
            raise ValueError("segments exceed the capacity")
        self.seg_off.copy_(off)

    def fit_models(self, stream=None):
        """PWL models of every window from the current sorted KPA (to be used
        on the next epoch's windows)."""
        K.kpa_pwl_fit(self.skeys, self.seg_off, 1024, models=self.models, stream=stream)

    def extract(self, rows, stream=None):
        """The step's first call alone: keys, row ids and the value column of
        the current rows (what the sort reads; an autotuner times sorts of
        them)."""
        K.kpa_extract(rows, self.layout, out_keys=self.keys, out_vals=self.vals, n=self.n,
                      stream=stream, with_rids=False)

    def step(self, rows, stream=None, cfg=None, fit_next=False):
        """Extract, batched sort, keyed reduction.  With fit_next, the step also
        fits each window's PWL model on its sorted KPA into next_models (the
        models the next epoch's windows would be sorted with); the models in
        use are not touched, so repeated steps do identical work."""
        cfg = self.cfg if cfg is None else cfg
        self.extract(rows, stream=stream)
        models = self.models if cfg.large_algo == K.KPA_SORT_LEARNED else None
        carry = self.carry if self.carry is not None else cfg.large_algo == K.KPA_SORT_LEARNED
        self.g = self._g[carry]
        if carry:
            K.kpa_batch_sort_vals(self.keys, None, self.vals, self.seg_off, cfg=cfg,
                                  n_cap=self.n, models=models, stats=self.stats,
                                  keys_out=self.skeys, rids_out=self.srids, vals_out=self.svals,
                                  ws=self.ws_sort, stream=stream)
        else:
            K.kpa_batch_sort(self.keys, None, self.seg_off, cfg=cfg, n_cap=self.n,
                             models=models, stats=self.stats, keys_out=self.skeys,
                             rids_out=self.srids, ws=self.ws_sort, stream=stream)
        outs = dict(self.g)
        outs["gkey"] = self.gkey
        outs["gseg_off"] = self.gseg
        if carry:   # values already in KPA order: no row ids to follow
            K.kpa_reduce_by_key(self.skeys, None, self.seg_off, self.svals, VALUE_COLUMN,
                                n_cap=self.n, want=self.want, ws=self.ws_red, stream=stream,
                                outs=outs)
        else:
            K.kpa_reduce_by_key(self.skeys, self.srids, self.seg_off, self.vals, VALUE_COLUMN,
                                n_cap=self.n, want=self.want, ws=self.ws_red, stream=stream,
                                outs=outs)
        if fit_next:
            K.kpa_pwl_fit(self.skeys, self.seg_off, 1024, models=self.next_models, stream=stream)

    def capture(self, rows, stream, cfg=None, fit_next=False):
        """A graph of one step on `stream` (replay with .launch())."""
        g = K.Graph.capture(stream)
        with g:
            self.step(rows, stream=stream, cfg=cfg, fit_next=fit_next)
        return g


class JoinMedian:
    """Temporal join and median per key of two streams over tumbling windows
    (Sec. 4.2 temporal join; Sec. 6 windowed median per key): each stream is
    partitioned into window KPAs (value column staged), each window's KPA is
    sorted, the lower median of every key is computed on both streams, and
    the two streams are merge-joined window by window (count and sum of
    value products mod 2^64).  The median pass also writes each key's count
    and sum of values, so the join intersects those two run lists
    (kpa_join_runs) and reads no value again; join_runs=False joins the
    sorted KPAs themselves (kpa_join), which reduces each side once more."""

    def __init__(self, n_l, n_r, layout, win_len, n_win, device="cuda", win_origin=0,
                 join_runs=True):
        self.n = (n_l, n_r)
        self.join_runs = join_runs
        self.layout, self.win_len, self.n_win, self.origin = layout, win_len, n_win, win_origin
        d = torch.device(device)
        i64 = dict(dtype=torch.int64, device=d)
        i32 = dict(dtype=torch.int32, device=d)
        u8 = dict(dtype=torch.uint8, device=d)
        self.side = []
        for n in self.n:
            cap = max(n, 1)
            sd = {
                "keys": torch.empty(cap, **i64), "rids": torch.empty(cap, **i32),
                "vals": torch.empty(cap, **i64), "skeys": torch.empty(cap, **i64),
                "srids": torch.empty(cap, **i32), "off": torch.empty(n_win + 1, **i64),
                "oob": torch.empty(1, **i64),
                "med": {"gkey": torch.empty(cap, **i64), "gmed": torch.empty(cap, **i64),
                        "gseg_off": torch.empty(n_win + 1, **i64)},
                "ws_part": torch.empty(K._ws_size("kpa_partition_windows_workspace_size", n,
                                                  n_win), **u8),
                "ws_sort": torch.empty(K.kpa_sort_workspace_size(n, n_win), **u8),
                "ws_med": torch.empty(K._ws_size("kpa_median_by_key_workspace_size", n, n_win),
                                      **u8),
            }
            if join_runs:  # each key's count and sum, written by the median pass
                sd["med"]["cnt"] = torch.empty(cap, **i64)
                sd["med"]["sum"] = torch.empty(cap, **i64)
            self.side.append(sd)
        jws = ("kpa_join_runs_workspace_size" if join_runs else "kpa_join_workspace_size")
        self.ws_join = torch.empty(K._ws_size(jws, n_l, n_r, n_win), **u8)
        self.join = {"count": torch.empty(n_win, **i64), "sumprod": torch.empty(n_win, **i64),
                     "npairs": torch.empty(1, **i64)}

    def step(self, rows_l, rows_r, stream=None):
        for sd, rows, n in zip(self.side, (rows_l, rows_r), self.n):
            K.kpa_partition_windows(rows, self.layout, self.win_len, self.n_win,
                                    win_origin=self.origin, n=n, out_keys=sd["keys"],
                                    out_rids=sd["rids"], out_win_off=sd["off"], out_oob=sd["oob"],
                                    ws=sd["ws_part"], stream=stream, out_vals=sd["vals"])
            K.kpa_sort_segmented(sd["keys"], sd["rids"], sd["off"], n_cap=n,
                                 keys_out=sd["skeys"], rids_out=sd["srids"], ws=sd["ws_sort"],
                                 stream=stream)
            K.kpa_median_by_key(sd["skeys"], sd["srids"], sd["off"], sd["vals"], VALUE_COLUMN,
                                n_cap=n, ws=sd["ws_med"], stream=stream, outs=sd["med"])
        L, R = self.side
        if self.join_runs:
            lm, rm = L["med"], R["med"]
            K.kpa_join_runs(lm["gkey"], lm["cnt"], lm["sum"], lm["gseg_off"], rm["gkey"],
                            rm["cnt"], rm["sum"], rm["gseg_off"], gl_cap=self.n[0],
                            gr_cap=self.n[1], ws=self.ws_join, stream=stream, outs=self.join)
        else:
            K.kpa_join(L["skeys"], L["srids"], L["off"], R["skeys"], R["srids"], R["off"],
                       L["vals"], R["vals"], VALUE_COLUMN, nl_cap=self.n[0], nr_cap=self.n[1],
                       ws=self.ws_join, stream=stream, outs=self.join)


class SlidingAggregation:
    """Per-key count, sum and max over sliding windows of length win_len that
    start every `slide` (win_len a multiple of slide; Sec. 4.2 "Windowing"
    partitions on the slide length).  A step partitions the rows into panes of
    one slide, sorts and reduces every pane once, then builds each window from
    its panes' groups (kpa_window_panes), sorts those by key and combines them:
    counts and sums add, maxima take the largest.  Window w covers
    [origin + w*slide, origin + w*slide + win_len), 0 <= w < n_win."""

    def __init__(self, n, layout, win_len, slide, n_win, device="cuda", win_origin=0):
        if win_len % slide:
            raise ValueError("win_len must be a multiple of slide")
        self.n, self.layout, self.slide, self.origin = n, layout, slide, win_origin
        self.P = win_len // slide
        self.n_win = n_win
        self.n_pane = n_win + self.P - 1
        d = torch.device(device)
        cap = max(n, 1)
        wcap = cap * self.P              # each pane group lies in at most P windows
        self.wcap = wcap
        i64 = dict(dtype=torch.int64, device=d)
        i32 = dict(dtype=torch.int32, device=d)
        u8 = dict(dtype=torch.uint8, device=d)
        self.pane = WindowAggregation(n, layout, slide, self.n_pane, k=1, device=device,
                                      win_origin=win_origin)
        self.cat_keys = torch.empty(wcap, **i64)
        self.cat_rids = torch.empty(wcap, **i32)
        self.cat_off = torch.empty(n_win + 1, **i64)
        self.s_keys = torch.empty(wcap, **i64)
        self.s_rids = torch.empty(wcap, **i32)
        self.ws_sort = torch.empty(K.kpa_sort_workspace_size(wcap, n_win), **u8)
        self.ws_red = torch.empty(K._ws_size("kpa_reduce_by_key_workspace_size", wcap, n_win),
                                  **u8)
        self.wkey = torch.empty(wcap, **i64)
        self.wseg = torch.empty(n_win + 1, **i64)
        self.w = {name: torch.empty(wcap, **i64) for name in ("cnt", "sum", "max")}
        self._scratch = {name: torch.empty(wcap, **i64) for name in ("cnt", "sum", "max")}

    def step(self, rows, stream=None):
        if self.n_pane > 256:
            raise ValueError("at most 256 panes")
        self.pane.step(rows, stream=stream)
        K.kpa_window_panes(self.pane.gkey, self.pane.gseg, self.P, self.wcap, stream=stream,
                           outs={"keys": self.cat_keys, "rids": self.cat_rids,
                                 "seg_off": self.cat_off})
        K.kpa_sort_segmented(self.cat_keys, self.cat_rids, self.cat_off, n_cap=self.wcap,
                             keys_out=self.s_keys, rids_out=self.s_rids, ws=self.ws_sort,
                             stream=stream)
        # one keyed reduction per pane column: sum of counts, sum of sums, max of maxima
        for col, want in (("cnt", "sum"), ("sum", "sum"), ("max", "max")):
            outs = {"gkey": self.wkey, "gseg_off": self.wseg, want: self.w[col]}
            K.kpa_reduce_by_key(self.s_keys, self.s_rids, self.cat_off, self.pane.g[col],
                                VALUE_COLUMN, n_cap=self.wcap, want=(want,), ws=self.ws_red,
                                stream=stream, outs=outs)


class AdPipeline:
    """The advertising pipeline of the paper's pipeline example (Sec. 4.3,
    shaped like the Yahoo streaming benchmark) on KPAs, over 32-byte rows
    {ad_id, event_type, ts, campaign slot}:

      Filter          Extract KPA(ad_id), Select the rows whose event type
                      (the value column) equals `keep_type`;
      External join   KeyUpdate: ad_id -> campaign in place from a small
                      sorted key-value table in device memory, then
                      write-back of the campaign into each row's slot;
      Window          KeySwap to the timestamp, Partition KPA(t) into
                      tumbling windows;
      Keyed agg.      KeySwap to the campaign, segmented sort, count per key.

    step() returns per-window (gkey, count, gseg_off) views and the number of
    ads missing from the table (their ad_id stays the key, as the update
    leaves them); rows are written (the campaign slot), as in the paper.
    The survivor count of the filter is read back to the host once per step
    (the later calls take it as their size)."""

    def __init__(self, n_rows, table_keys, table_vals, win_len, n_win, keep_type=0,
                 device="cuda", win_origin=0):
        from datagen.rows import LAYOUT_YSB, YSB_COLS
        self.n, self.win_len, self.n_win, self.origin = n_rows, win_len, n_win, win_origin
        self.layout, self.cols = LAYOUT_YSB, YSB_COLS
        self.tk, self.tv = table_keys, table_vals
        d = torch.device(device)
        cap = max(n_rows, 1)
        i64 = dict(dtype=torch.int64, device=d)
        i32 = dict(dtype=torch.int32, device=d)
        self.keys = torch.empty(cap, **i64)
        self.rids = torch.empty(cap, **i32)
        self.fkeys = torch.empty(cap, **i64)
        self.frids = torch.empty(cap, **i32)
        self.pkeys = torch.empty(cap, **i64)
        self.prids = torch.empty(cap, **i32)
        self.skeys = torch.empty(cap, **i64)
        self.srids = torch.empty(cap, **i32)
        self.gkey = torch.empty(cap, **i64)
        self.gcnt = torch.empty(cap, **i64)
        self.one_seg = torch.tensor([0, n_rows], **i64)
        self.foff = torch.empty(2, **i64)
        self.woff = torch.empty(n_win + 1, **i64)
        self.oob = torch.empty(1, **i64)
        self.gseg = torch.empty(n_win + 1, **i64)
        self.missing = torch.empty(1, **i64)
        self.keep = torch.tensor([keep_type], **i64)
        u8 = dict(dtype=torch.uint8, device=d)
        self.ws_sel = torch.empty(K._ws_size("kpa_select_workspace_size", n_rows, 1), **u8)
        self.ws_part = torch.empty(K._ws_size("kpa_partition_windows_workspace_size", n_rows,
                                              n_win), **u8)
        self.ws_sort = torch.empty(K.kpa_sort_workspace_size(n_rows, n_win), **u8)
        self.ws_red = torch.empty(K._ws_size("kpa_reduce_by_key_workspace_size", n_rows, n_win),
                                  **u8)

    def step(self, rows, stream=None):
        L, c = self.layout, self.cols
        K.kpa_extract(rows, L, out_keys=self.keys, out_rids=self.rids, n=self.n, stream=stream)
        K.kpa_select(self.keys, self.rids, self.one_seg, self.keep, op="==",
                     column=K.KPA_SEL_VALUE, rows=rows, layout=L, n_cap=self.n,
                     outs={"keys": self.fkeys, "rids": self.frids, "seg_off": self.foff},
                     ws=self.ws_sel, stream=stream)
        m = int(self.foff[1].item())       # survivors: the size of every later call
        K.kpa_key_update(self.fkeys, self.tk, self.tv, n=m, out_missing=self.missing,
                         stream=stream)
        K.kpa_key_writeback(self.fkeys, self.frids, rows, 32, c["campaign"], n=m, stream=stream)
        tkeys = K.kpa_keyswap(self.frids[:m], rows, 32, c["ts"], out_keys=self.fkeys,
                              stream=stream)
        K.kpa_partition_kpa(tkeys, self.frids, self.win_len, self.n_win, self.origin, n=m,
                            out_keys=self.pkeys, out_rids=self.prids, out_win_off=self.woff,
                            out_oob=self.oob, ws=self.ws_part, stream=stream)
        p = int(self.woff[-1].item())      # entries inside the windows
        K.kpa_keyswap(self.prids[:p], rows, 32, c["campaign"], out_keys=self.pkeys,
                      stream=stream)
        K.kpa_sort_segmented(self.pkeys, self.prids, self.woff, n_cap=max(p, 1),
                             keys_out=self.skeys, rids_out=self.srids, ws=self.ws_sort,
                             stream=stream)
        K.kpa_reduce_by_key(self.skeys, self.srids, self.woff, None, None, n_cap=max(p, 1),
                            want=("cnt",), ws=self.ws_red, stream=stream,
                            outs={"gkey": self.gkey, "cnt": self.gcnt, "gseg_off": self.gseg})
        return {"survivors": m, "in_windows": p}
