"""Host logic of the counter summary (paper_2409_08090_amd.traffic): which
dispatch of a periodogram counts toward which stage, on a synthetic trace."""
from paper_2409_08090_amd import traffic


def _step(scale=1.0):
    names = [
        ("void mils::k_stats(mils::CallArgs, mils::Work)", 1),
        ("void mils::k_stats_final(mils::CallArgs, mils::Work, int)", 1),
        ("void mils::k_bins_sorted(mils::CallArgs, mils::Plan, mils::Work)", 2),
        ("void mils::k_lowfreq(mils::CallArgs, mils::Work)", 3),
        ("void mils::k_lowfreq_final(mils::CallArgs, mils::Work, int)", 1),
        ("void mils::k_row_flags(mils::Plan, mils::Work, int, int)", 1),
        ("void mils::k_spread_rows<double, 2, 1>(mils::CallArgs, mils::Plan, mils::Work)", 5),
        ("void mils::k_row_compact(mils::Plan, mils::Work, int)", 1),
        ("void mils::k_spread_rows<double, 1, 2>(mils::CallArgs, mils::Plan, mils::Work)", 7),
        ("void mils::k_fft_pass<double, 2048, 256, false>(...)", 11),   # first pass, 2f grid
        ("void mils::k_fft_pass<double, 2048, 256, false>(...)", 13),   # first pass, f grids
        ("void mils::k_fft_pass<double, 2048, 256, false>(...)", 17),   # middle pass
        ("void mils::k_fft_last<double, 3, 3072, 256, false>(...)", 19),
    ]
    return [(0, n, k * scale) for n, k in names]


def test_stage_bytes_per_periodogram():
    disp = [(0, "void mils::k_phihat(...)", 100.0)] + _step() + _step(3.0)
    got = traffic.stage_bytes(disp, 1.0 / 1024.0)
    # the average of the two periodograms (scales 1 and 3)
    want = {"stats": 2, "bin_sort": 2, "lowfreq": 4, "spread_2f": 5, "spread_f": 7,
            "row_class": 2, "fft_pass_0": 24, "fft_pass_1": 17, "fft_last_power": 19}
    assert set(got) == set(want)
    for k, v in want.items():
        assert abs(got[k] - 2.0 * v) < 1e-9, k


def test_incomplete_periodogram_is_ignored():
    disp = _step() + _step(5.0)[:6]
    got = traffic.stage_bytes(disp, 1.0 / 1024.0)
    assert abs(got["fft_pass_1"] - 17.0) < 1e-9
    assert abs(got["stats"] - 2.0) < 1e-9


def test_spread_names_with_more_template_arguments():
    step = [(0, n.replace("<double, 2, 1>", "<double, 2, 1, false>")
             .replace("<double, 1, 2>", "<double, 1, 2, false>"), k) for _, n, k in _step()]
    got = traffic.stage_bytes(step, 1.0 / 1024.0)
    assert abs(got["spread_2f"] - 5.0) < 1e-9 and abs(got["fft_pass_0"] - 24.0) < 1e-9


def test_copy_scale():
    disp = [(0, "__amd_rocclr_copyBuffer", traffic.COPY_BYTES / 1024.0 / 2.0)]
    assert abs(traffic.copy_scale(disp) - 2.0) < 1e-12
    assert traffic.copy_scale([(0, "k_stats", 1.0)]) is None


def test_two_pass_plan_stages():
    step = [
        ("void mils::k_stats(mils::CallArgs, mils::Work)", 1),
        ("void mils::k_bins_sorted(mils::CallArgs, mils::Plan, mils::Work)", 2),
        ("void mils::k_row_compact(mils::Plan, mils::Work, int)", 1),
        ("void mils::k_row_flags(mils::Plan, mils::Work, int, int)", 1),
        ("void mils::k_spread_rows<double, 1, 2, false>(mils::CallArgs, mils::Plan, mils::Work)", 7),
        ("void mils::k_spread_rows<double, 2, 1, false>(mils::CallArgs, mils::Plan, mils::Work)", 5),
        ("void mils::k_fft2_first<double, 4096, 4, true>(...)", 30),
        ("void mils::k_lowfreq(mils::CallArgs, mils::Work)", 3),
        ("void mils::k_fft2_last<double, 4096, 3, 4, true>(...)", 40),
        ("void mils::k_fft2_out<double, 64>(...)", 6),
    ]
    got = traffic.stage_bytes([(0, n, k) for n, k in step], 1.0 / 1024.0)
    want = {"stats": 1, "bin_sort": 2, "row_class": 2, "spread_f": 7, "spread_2f": 5,
            "fft_pass_0": 30, "lowfreq": 3, "fft_last_power": 40, "fft_out": 6}
    assert got == {k: float(v) for k, v in want.items()}


def test_kernel_counters_summary(tmp_path):
    hdr = ('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value","Start_Timestamp",'
           '"End_Timestamp"\n')
    rows = []
    for did, (w, v, wc, la, bc) in enumerate([(4, 100, 1000, 50, 5), (4, 300, 3000, 150, 15)]):
        name = '"void mils::k_fft2_last<double, 4096, 3, 4, true>(mils::Fft2Bufs<double>)"'
        for cn, val in (("SQ_WAVES", w), ("SQ_INSTS_VALU", v), ("SQ_WAVE_CYCLES", wc),
                        ("SQ_LDS_IDX_ACTIVE", la), ("SQ_LDS_BANK_CONFLICT", bc)):
            rows.append(f'{did},{name},"{cn}",{val},1000,{1000 + 100 * (did + 1)}\n')
    d = tmp_path / "run"
    d.mkdir()
    (d / "x_counter_collection.csv").write_text(hdr + "".join(rows))
    got = traffic.kernel_counters([str(d)], cycles_per_ns=1.0, num_cu=1)
    e = got["k_fft2_last<double, 4096, 3, 4, true>"]
    assert e["dispatches"] == 2 and e["mean_ns"] == 150.0
    assert e["SQ_INSTS_VALU"] == 200.0 and e["valu_per_wave"] == 50.0
    assert abs(e["bank_conflict"] - 0.1) < 1e-12
    assert abs(e["lds_util"] - 100.0 / 150.0) < 1e-12


def test_short_names():
    assert traffic.short_name(
        '"void mils::(anonymous namespace)::k_bpass<double>(mils::BatchArgs, int)"') == \
        "k_bpass<double>"
    assert traffic.short_name("mils::k_stats(mils::CallArgs, mils::Work)") == "k_stats"
