"""The build's matrix-core accumulator check (paper_1209_4297_amd/build.py): an MFMA whose
accumulator source is not its destination must not have that source overwritten by a non-MFMA
instruction shortly after it.  Synthetic gfx950 assembly exercises each rule."""
from paper_1209_4297_amd.build import MFMA_WAR_WINDOW, mfma_accumulator_hazards


def _asm(*lines):
    return "k:\n" + "\n".join("\t" + l for l in lines) + "\n"


def test_lds_load_into_a_renamed_accumulator_source_is_flagged():
    asm = _asm("v_mfma_f32_16x16x32_bf16 v[138:141], v[158:161], v[190:193], v[106:109]",
               "s_nop 2",
               "ds_read_b128 v[106:109], v208 offset:30720")
    hits = mfma_accumulator_hazards(asm)
    assert len(hits) == 1 and hits[0][3].startswith("ds_read_b128")


def test_valu_write_of_a_partial_source_register_is_flagged():
    asm = _asm("v_mfma_f64_16x16x4_f64 v[2:9], v[20:21], v[22:23], v[30:37]",
               "v_add_f64 v[36:37], v[40:41], v[42:43]")
    assert len(mfma_accumulator_hazards(asm)) == 1


def test_in_place_accumulation_is_not_flagged():
    asm = _asm("v_mfma_f32_16x16x32_bf16 v[2:5], v[70:73], v[102:105], v[2:5]",
               "ds_read_b128 v[2:5], v207")
    assert mfma_accumulator_hazards(asm) == []


def test_later_mfma_writing_the_source_is_not_flagged():
    # the matrix core executes MFMAs in order: a later MFMA cannot write before an earlier reads
    asm = _asm("v_mfma_f32_16x16x4_f32 a[56:59], v130, v146, a[60:63]",
               "v_mfma_f32_16x16x4_f32 a[60:63], v131, v147, a[64:67]")
    assert mfma_accumulator_hazards(asm) == []


def test_writer_beyond_the_window_and_stores_are_not_flagged():
    asm = _asm("v_mfma_f32_16x16x32_bf16 v[138:141], v[158:161], v[190:193], v[106:109]",
               "ds_write_b128 v1, v[106:109]",
               *(["s_nop 0"] * MFMA_WAR_WINDOW),
               "ds_read_b128 v[106:109], v208")
    assert mfma_accumulator_hazards(asm) == []


def test_functions_are_scanned_separately():
    asm = ("f:\n\tv_mfma_f32_16x16x32_bf16 v[8:11], v[0:3], v[4:7], v[12:15]\n"
           "g:\n\tds_read_b128 v[12:15], v1\n")
    assert mfma_accumulator_hazards(asm) == []
