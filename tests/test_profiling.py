"""Host logic of the profile summaries: the source digest that ties a traffic
summary to the kernels it was measured on."""

import os

from paper_2003_03931_amd import profiling


def _tree(tmp_path, name, text):
    d = tmp_path / name / "csrc"
    d.mkdir(parents=True)
    (d / "k.hip").write_text(text)
    (d / "pp.hip").write_text("int not_in_step;\n")
    return str(tmp_path / name)


def test_digest_ignores_comments_and_blank_lines(tmp_path):
    a = _tree(tmp_path, "a", "int x = 1;  // one\n\n/* block\n   comment */\nint y;\n")
    b = _tree(tmp_path, "b", "int x = 1;\n// another comment\nint y;   \n")
    assert profiling.source_digest(a) == profiling.source_digest(b)


def test_digest_follows_code_changes(tmp_path):
    a = _tree(tmp_path, "a", "int x = 1;\n")
    b = _tree(tmp_path, "b", "int x = 2;\n")
    assert profiling.source_digest(a) != profiling.source_digest(b)


def test_digest_skips_sources_outside_the_step(tmp_path):
    a = _tree(tmp_path, "a", "int x = 1;\n")
    with open(os.path.join(a, "csrc", "pp.hip"), "w") as f:
        f.write("int changed;\n")
    b = _tree(tmp_path, "b", "int x = 1;\n")
    assert profiling.source_digest(a) == profiling.source_digest(b)
